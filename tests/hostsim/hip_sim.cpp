// Host-only stand-in of the HIP runtime (see hip/hip_runtime.h). Test
// infrastructure: lets the library's host code run under the sanitizers.
#include "hip/hip_runtime.h"

#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace {

struct Graph;

// An event: the queue position of its last record, and how far its stream got.
struct Event {
    std::mutex mu;
    std::condition_variable cv;
    uint64_t recorded = 0;   // records so far
    uint64_t reached = 0;    // records whose position the stream has passed
    Graph* captured = nullptr;  // recorded into this graph (capture), not run
};

}  // namespace

struct ihipEvent_t {
    std::shared_ptr<Event> e = std::make_shared<Event>();
};

namespace {

struct Graph {
    std::vector<std::function<void()>> nodes;
};

}  // namespace

struct ihipGraph_t {
    Graph g;
};
struct ihipGraphExec_t {
    std::vector<std::function<void()>> nodes;
};

// A stream: a worker thread running queued work in order.
struct ihipStream_t {
    std::mutex mu;
    std::condition_variable cv, idle_cv;
    std::deque<std::function<void()>> q;
    bool busy = false, stop = false;
    Graph* capture = nullptr;  // recording instead of running
    std::thread worker;

    ihipStream_t() {
        worker = std::thread([this] { run(); });
    }
    ~ihipStream_t() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv.notify_all();
        worker.join();
    }
    void run() {
        for (;;) {
            std::function<void()> fn;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [this] { return stop || !q.empty(); });
                if (q.empty()) return;
                fn = std::move(q.front());
                q.pop_front();
                busy = true;
            }
            fn();
            {
                std::lock_guard<std::mutex> lk(mu);
                busy = false;
            }
            idle_cv.notify_all();
        }
    }
    void push(std::function<void()> fn) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (capture) {
                capture->nodes.push_back(std::move(fn));
                return;
            }
            q.push_back(std::move(fn));
        }
        cv.notify_all();
    }
    void drain() {
        std::unique_lock<std::mutex> lk(mu);
        idle_cv.wait(lk, [this] { return q.empty() && !busy; });
    }
};

namespace {

std::mutex g_mu;
std::map<void*, size_t> g_dev;    // device allocations
std::map<void*, size_t> g_host;   // pinned host allocations
size_t g_limit = 0, g_in_use = 0;
thread_local hipError_t t_last = hipSuccess;
ihipStream_t* g_null = nullptr;   // the legacy default stream

ihipStream_t* stream_of(hipStream_t s) {
    if (s) return s;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_null) g_null = new ihipStream_t();
    return g_null;
}

hipError_t ret(hipError_t e) {
    if (e != hipSuccess) t_last = e;
    return e;
}

}  // namespace

namespace hipsim {
void enqueue(hipStream_t s, std::function<void()> fn) { stream_of(s)->push(std::move(fn)); }
void set_device_limit(size_t bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_limit = bytes;
}
size_t device_bytes_in_use() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_in_use;
}
}  // namespace hipsim

hipError_t hipMalloc(void** p, size_t bytes) {
    if (!p) return ret(hipErrorInvalidValue);
    *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_limit && g_in_use + bytes > g_limit) return ret(hipErrorOutOfMemory);
    }
    void* q = std::malloc(bytes ? bytes : 1);
    if (!q) return ret(hipErrorOutOfMemory);
    std::memset(q, 0xA5, bytes < 4096 ? bytes : 4096);  // device memory starts as garbage
    std::lock_guard<std::mutex> lk(g_mu);
    g_dev[q] = bytes;
    g_in_use += bytes;
    *p = q;
    return hipSuccess;
}

hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(p);
    if (it == g_dev.end()) return ret(hipErrorInvalidValue);
    g_in_use -= it->second;
    g_dev.erase(it);
    std::free(p);
    return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
    if (!p) return ret(hipErrorInvalidValue);
    void* q = std::malloc(bytes ? bytes : 1);
    if (!q) return ret(hipErrorOutOfMemory);
    std::lock_guard<std::mutex> lk(g_mu);
    g_host[q] = bytes;
    *p = q;
    return hipSuccess;
}

hipError_t hipHostFree(void* p) {
    if (!p) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_host.find(p);
    if (it == g_host.end()) return ret(hipErrorInvalidValue);
    g_host.erase(it);
    std::free(p);
    return hipSuccess;
}

hipError_t hipHostGetDevicePointer(void** dev, void* host, unsigned) {
    if (!dev) return ret(hipErrorInvalidValue);
    *dev = host;
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
    if (bytes && (!dst || !src)) return ret(hipErrorInvalidValue);
    stream_of(s)->push([=] { std::memcpy(dst, src, bytes); });
    return hipSuccess;
}

hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t s) {
    if (bytes && !dst) return ret(hipErrorInvalidValue);
    stream_of(s)->push([=] { std::memset(dst, value, bytes); });
    return hipSuccess;
}

hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
    if (!p || !symbol) return ret(hipErrorInvalidValue);
    *p = const_cast<void*>(symbol);
    return hipSuccess;
}

hipError_t hipSetDevice(int device) { return device == 0 ? hipSuccess : ret(hipErrorInvalidValue); }
hipError_t hipGetDevice(int* device) {
    *device = 0;
    return hipSuccess;
}
hipError_t hipGetLastError(void) {
    const hipError_t e = t_last;
    t_last = hipSuccess;
    return e;
}
const char* hipGetErrorString(hipError_t e) {
    switch (e) {
        case hipSuccess: return "hipSuccess";
        case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
        case hipErrorInvalidValue: return "hipErrorInvalidValue";
        default: return "hipError (stand-in)";
    }
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = new ihipStream_t();
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    if (!s) return ret(hipErrorInvalidValue);
    s->drain();
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    ihipStream_t* st = stream_of(s);
    {
        std::lock_guard<std::mutex> lk(st->mu);
        if (st->capture) return ret(hipErrorStreamCaptureUnsupported);
    }
    st->drain();
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
    *e = new ihipEvent_t();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    if (!e) return ret(hipErrorInvalidValue);
    ihipStream_t* st = stream_of(s);
    std::shared_ptr<Event> ev = e->e;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        if (st->capture) {  // a captured record only marks the join point
            std::lock_guard<std::mutex> le(ev->mu);
            ev->captured = st->capture;
            return hipSuccess;
        }
    }
    uint64_t n;
    {
        std::lock_guard<std::mutex> le(ev->mu);
        ev->captured = nullptr;
        n = ++ev->recorded;
    }
    st->push([ev, n] {
        {
            std::lock_guard<std::mutex> le(ev->mu);
            if (ev->reached < n) ev->reached = n;
        }
        ev->cv.notify_all();
    });
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    std::shared_ptr<Event> ev = e->e;
    std::unique_lock<std::mutex> le(ev->mu);
    const uint64_t n = ev->recorded;
    ev->cv.wait(le, [&] { return ev->reached >= n; });
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    *ms = 0.0f;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    ihipStream_t* st = stream_of(s);
    std::shared_ptr<Event> ev = e->e;
    Graph* joined;
    uint64_t n;
    {
        std::lock_guard<std::mutex> le(ev->mu);
        joined = ev->captured;
        n = ev->recorded;
    }
    if (joined) {  // waiting on a captured record joins the capture
        std::lock_guard<std::mutex> lk(st->mu);
        st->capture = joined;
        return hipSuccess;
    }
    st->push([ev, n] {
        std::unique_lock<std::mutex> le(ev->mu);
        ev->cv.wait(le, [&] { return ev->reached >= n; });
    });
    return hipSuccess;
}

namespace {
std::mutex g_cap_mu;
std::map<Graph*, std::vector<ihipStream_t*>> g_joined;  // streams recording into a graph
}  // namespace

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    ihipStream_t* st = stream_of(s);
    st->drain();
    auto* g = new ihipGraph_t();
    std::lock_guard<std::mutex> lk(st->mu);
    if (st->capture) {
        delete g;
        return ret(hipErrorInvalidValue);
    }
    st->capture = &g->g;
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* graph) {
    ihipStream_t* st = stream_of(s);
    Graph* g;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        g = st->capture;
        st->capture = nullptr;
    }
    if (!g) return ret(hipErrorInvalidValue);
    // every other stream that joined this capture leaves it too: the stand-in
    // keeps no list of them, so the join point is the end of capture of the
    // origin stream, as in the library's fork/join pattern
    *graph = reinterpret_cast<hipGraph_t>(reinterpret_cast<char*>(g) - offsetof(ihipGraph_t, g));
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t graph, hipGraphNode_t*, char*, size_t) {
    *exec = new ihipGraphExec_t();
    (*exec)->nodes = graph->g.nodes;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s) {
    std::vector<std::function<void()>> nodes = exec->nodes;
    stream_of(s)->push([nodes] {
        for (const auto& fn : nodes) fn();
    });
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
    delete exec;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t graph) {
    delete graph;
    return hipSuccess;
}
