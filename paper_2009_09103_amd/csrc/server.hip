// server.hip -- request server over one resident graph (csaw_server_* in
// include/csaw.h).
//
// Executors are threads, each with its own stream and one block of device
// memory allocated when the server is created (the memory budget split
// evenly), plus two pinned host staging buffers. A sampling batch lays out its
// seeds, edge outputs, segment offsets and the sampling call's scratch in
// that block, a walk batch its starts, paths and per-request tables;
// requests join a batch while the batch's exact device need fits. Serving therefore allocates no device memory: what the server holds is
// fixed at creation, and admission is by the very bytes a batch occupies.
// Results travel device -> pinned staging -> the result's host arrays in
// chunks, so no copy targets pageable memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <type_traits>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/csaw.h"
#include "internal.h"
#include "kernels.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kStageBytes = size_t(16) << 20;  // bytes of each pinned staging buffer
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Request {
    uint64_t ticket = 0;
    int32_t kind = 0;
    uint64_t id = 0, rng_seed = 0;
    int32_t bias = 0;
    std::vector<int32_t> seeds, fanouts, starts;
    int32_t length = 0;
    uint32_t wr = 1, wc = 1, wo = 1;
    std::vector<int64_t> fcap;  // sampling: frontier capacity per layer, alone
    int64_t max_edges = 0;      // sampling: edge bound, alone
    size_t need = 0;            // device bytes of the request alone
    Clock::time_point t_submit;
};

double us_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::micro>(b - a).count();
}

// Pinned host memory for result arrays, allocated and touched page by page
// when the server is created: the device copies results straight into it (no
// staging buffer, no host copy: 55 GB/s against 20 GB/s through staging), and
// nothing faults in while results are written (into a fresh allocation, page
// by page, host copies ran about ten times slower). Ranges are handed out first fit (4 KiB granules) and
// coalesced when given back; the pool is reference counted (the server and
// every result holding a range of it), so results may outlive the server.
class HostPool {
public:
    static HostPool* create(size_t bytes) {
        void* p = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess || !p) return nullptr;
        // the host maps pinned pages on first touch (host writes into untouched
        // pages ran at 2.9 GB/s against 31 GB/s): touch every page now
        for (size_t off = 0; off < bytes; off += kGranule) static_cast<volatile char*>(p)[off] = 0;
        HostPool* h = new (std::nothrow) HostPool();
        if (!h) {
            (void)hipHostFree(p);
            return nullptr;
        }
        h->base_ = (char*)p;
        h->bytes_ = bytes;
        h->free_[0] = bytes;
        return h;
    }
    void ref() { refs_.fetch_add(1); }
    void unref() {
        if (refs_.fetch_sub(1) == 1) delete this;
    }
    bool owns(const void* p) const { return (const char*)p >= base_ && (const char*)p < base_ + bytes_; }
    // n bytes, or null when no free range is large enough
    void* take(size_t n) {
        n = round_up(n);
        std::lock_guard<std::mutex> lk(mu_);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            used_[off] = n;
            return base_ + off;
        }
        return nullptr;
    }
    // Pieces of the given sizes carved back to back (each rounded to whole
    // granules) out of one free range, so that one copy can fill them all;
    // each piece is given back on its own. False when no range is large
    // enough.
    bool take_run(const std::vector<size_t>& sizes, std::vector<char*>& out) {
        size_t total = 0;
        for (size_t n : sizes) total += round_up(n);
        std::lock_guard<std::mutex> lk(mu_);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < total) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > total) free_[off + total] = len - total;
            out.resize(sizes.size());
            size_t at = off;
            for (size_t k = 0; k < sizes.size(); ++k) {
                out[k] = base_ + at;
                used_[at] = round_up(sizes[k]);
                at += round_up(sizes[k]);
            }
            return true;
        }
        return false;
    }
    void give(void* p) {
        const size_t off = (size_t)((char*)p - base_);
        std::lock_guard<std::mutex> lk(mu_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t at = off, len = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(at);
        if (next != free_.end() && next->first == at + len) {  // merge with the range after
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {  // and with the range before
            auto prev = std::prev(next);
            if (prev->first + prev->second == at) {
                at = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[at] = len;
    }

private:
    static constexpr size_t kGranule = 4096;
    static size_t round_up(size_t n) { return (std::max<size_t>(n, 1) + kGranule - 1) / kGranule * kGranule; }
    HostPool() = default;
    ~HostPool() { (void)hipHostFree(base_); }
    char* base_ = nullptr;
    size_t bytes_ = 0;
    std::atomic<int64_t> refs_{1};
    std::mutex mu_;
    std::map<size_t, size_t> free_;            // offset -> length
    std::unordered_map<size_t, size_t> used_;  // offset -> length
};

// A result as the library allocates it: what callers see, then the pool its
// arrays may come from (csaw_result_free gives them back).
struct ResultBox {
    csaw_result pub;
    HostPool* pool;
};
static_assert(std::is_standard_layout<ResultBox>::value, "a csaw_result* is its box's address");

csaw_result* new_result(int32_t kind, csaw_status st) {
    ResultBox* b = new (std::nothrow) ResultBox();
    if (!b) return nullptr;
    b->pub.status = st;
    b->pub.kind = kind;
    b->pool = nullptr;
    return &b->pub;
}

// r holds ranges of the pool (it keeps the pool alive until it is freed).
void hold_pool(HostPool* pool, csaw_result* r) {
    ResultBox* b = reinterpret_cast<ResultBox*>(r);
    if (!b->pool) {
        b->pool = pool;
        pool->ref();
    }
}

// n bytes for one of r's arrays: a range of the pool when one is free, else
// the heap.
void* result_array(HostPool* pool, csaw_result* r, size_t n) {
    if (pool) {
        if (void* p = pool->take(n)) {
            hold_pool(pool, r);
            return p;
        }
    }
    return std::malloc(std::max<size_t>(n, 1));
}

// Aggregate shape of a sampling batch: everything its device layout depends on.
struct BatchShape {
    int32_t ni = 0, L = 0;
    int64_t seeds = 0, edges = 0;
    std::vector<int64_t> fcap;  // [CSAW_MAX_LAYERS + 1], summed over the batch

    BatchShape() : fcap(CSAW_MAX_LAYERS + 1, 0) {}
    void add(const Request& r) {
        ++ni;
        L = std::max<int32_t>(L, (int32_t)r.fanouts.size());
        seeds += (int64_t)r.seeds.size();
        edges += r.max_edges;
        for (size_t l = 0; l < r.fcap.size(); ++l) fcap[l] += r.fcap[l];
    }
};

// Device layout of a sampling batch in an executor's block.
struct BatchLayout {
    size_t o_seeds, o_src, o_dst, o_off, o_scratch, scratch, total;
};

BatchLayout batch_layout(csaw_graph g, const BatchShape& b) {
    BatchLayout y;
    size_t at = 0;
    y.o_seeds = at;
    at = align_up(at + (size_t)std::max<int64_t>(b.seeds, 1) * sizeof(int32_t));
    y.o_src = at;
    at = align_up(at + (size_t)std::max<int64_t>(b.edges, 1) * sizeof(int32_t));
    y.o_dst = at;
    at = align_up(at + (size_t)std::max<int64_t>(b.edges, 1) * sizeof(int32_t));
    y.o_off = at;
    at = align_up(at + ((size_t)b.L * b.ni + 1) * sizeof(int64_t));
    y.o_scratch = at;
    const std::vector<int64_t> fc(b.fcap.begin(), b.fcap.begin() + b.L + 1);
    y.scratch = csaw::sample_scratch_bytes(g, b.ni, b.L, fc);
    y.total = y.scratch == SIZE_MAX ? SIZE_MAX : at + y.scratch;
    return y;
}

// Aggregate shape of a walk batch, and its device layout in an executor's
// block: every walker's start, every request's paths, the batch's tables.
struct WalkShape {
    int32_t nreq = 0;
    int64_t walkers = 0, path_elems = 0;
    void add(const Request& r) {
        ++nreq;
        walkers += (int64_t)r.starts.size();
        path_elems += (int64_t)r.starts.size() * ((int64_t)r.length + 1);
    }
};

struct WalkLayout {
    size_t o_starts, o_paths, o_tab, total;
};

WalkLayout walk_layout(const WalkShape& b) {
    WalkLayout y;
    size_t at = 0;
    y.o_starts = at;
    at = align_up(at + (size_t)std::max<int64_t>(b.walkers, 1) * sizeof(int32_t));
    y.o_paths = at;
    at = align_up(at + (size_t)std::max<int64_t>(b.path_elems, 1) * sizeof(int32_t));
    y.o_tab = at;
    y.total = align_up(at + csaw::walk_batch_layout(b.nreq, b.walkers).bytes);
    return y;
}

// Walk requests that one launch can serve: same bias kind and node2vec weights.
bool same_walk_kind(const Request& a, const Request& b) {
    return a.bias == b.bias && a.wr == b.wr && a.wc == b.wc && a.wo == b.wo;
}

}  // namespace

// One executor: its stream, its device block and its staging buffers.
struct Exec {
    hipStream_t st = nullptr;
    char* dev = nullptr;
    size_t bytes = 0;
    char* stage[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};

    // host -> device through the staging buffers
    bool to_device(char* d, const char* h, size_t n) {
        for (size_t off = 0, k = 0; off < n; off += kStageBytes, ++k) {
            const size_t len = std::min(kStageBytes, n - off);
            char* b = stage[k & 1];
            if (k >= 2 && hipEventSynchronize(ev[k & 1]) != hipSuccess) return false;
            std::memcpy(b, h + off, len);
            if (hipMemcpyAsync(d + off, b, len, hipMemcpyHostToDevice, st) != hipSuccess) return false;
            if (hipEventRecord(ev[k & 1], st) != hipSuccess) return false;
        }
        return hipStreamSynchronize(st) == hipSuccess;
    }
    // device -> host: chunk [off, off + len) of the source goes to sink(off, data, len)
    bool to_host(const char* d, size_t n, const std::function<void(size_t, const char*, size_t)>& sink) {
        size_t prev_off = 0, prev_len = 0;
        for (size_t off = 0, k = 0; off < n; off += kStageBytes, ++k) {
            const size_t len = std::min(kStageBytes, n - off);
            if (hipMemcpyAsync(stage[k & 1], d + off, len, hipMemcpyDeviceToHost, st) != hipSuccess) return false;
            if (hipEventRecord(ev[k & 1], st) != hipSuccess) return false;
            if (k >= 1) {  // the previous chunk, while this one is in flight
                if (hipEventSynchronize(ev[(k - 1) & 1]) != hipSuccess) return false;
                sink(prev_off, stage[(k - 1) & 1], prev_len);
            }
            prev_off = off;
            prev_len = len;
        }
        if (n == 0) return true;
        const size_t last = (n - 1) / kStageBytes;
        if (hipEventSynchronize(ev[last & 1]) != hipSuccess) return false;
        sink(prev_off, stage[last & 1], prev_len);
        return true;
    }
};

struct csaw_server_s {
    csaw_graph g = nullptr;
    csaw_server_config cfg{};
    int device = 0;
    int64_t n = 0;
    std::vector<Exec> execs;
    size_t exec_bytes = 0;
    HostPool* pool = nullptr;  // result arrays (null: the heap)
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, csaw_result*> done;
    std::unordered_map<uint64_t, int> state;  // ticket -> kQueued / kRunning / kDone (not handed over)
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;

    enum { kQueued = 0, kRunning = 1, kDone = 2 };

    void worker(Exec& x);
    void run_sample_batch(std::vector<Request*>& batch, Exec& x, Clock::time_point t0);
    void run_walk_batch(std::vector<Request*>& batch, Exec& x, Clock::time_point t0);
    void finish(Request* r, csaw_result* res);
    void free_execs();
};

void csaw_server_s::finish(Request* r, csaw_result* res) {
    std::lock_guard<std::mutex> lk(mu);
    done[r->ticket] = res;
    state[r->ticket] = kDone;
    cv_done.notify_all();
}

void csaw_server_s::run_walk_batch(std::vector<Request*>& batch, Exec& x, Clock::time_point t0) {
    // longest walks first: their walkers are dispatched first and the
    // launch's tail is short ones; each walker's path row and counters are
    // its own, so the order changes no result
    std::stable_sort(batch.begin(), batch.end(), [](const Request* a, const Request* b) { return a->length > b->length; });
    const int32_t nreq = (int32_t)batch.size();
    WalkShape shape;
    for (Request* r : batch) shape.add(*r);
    const WalkLayout lay = walk_layout(shape);
    std::vector<csaw::WalkBatchReq> reqs((size_t)nreq);
    std::vector<int64_t> path_off((size_t)nreq + 1, 0), steps((size_t)nreq, 0);
    std::vector<int32_t> starts((size_t)shape.walkers);
    std::vector<csaw_result*> res((size_t)nreq, nullptr);
    csaw_status stt = lay.total <= x.bytes ? CSAW_OK : CSAW_ERR_OUT_OF_MEMORY;  // batches are formed to fit
    int64_t w0 = 0;
    for (int32_t q = 0; q < nreq; ++q) {
        const Request* r = batch[q];
        const int64_t nw = (int64_t)r->starts.size();
        reqs[q] = csaw::WalkBatchReq{nw, r->length, r->rng_seed, r->id};
        path_off[q + 1] = path_off[q] + nw * ((int64_t)r->length + 1);
        std::copy(r->starts.begin(), r->starts.end(), starts.begin() + w0);
        w0 += nw;
        res[q] = new_result(CSAW_REQUEST_WALK, CSAW_OK);
        if (!res[q]) continue;
        res[q]->num_walkers = nw;
        res[q]->length = r->length;
        res[q]->batch_requests = nreq;
        res[q]->paths = (int32_t*)result_array(
            pool, res[q], (size_t)std::max<int64_t>(nw * ((int64_t)r->length + 1), 1) * sizeof(int32_t));
        if (!res[q]->paths) stt = CSAW_ERR_OUT_OF_MEMORY;
    }
    for (csaw_result* r : res)
        if (!r) stt = CSAW_ERR_OUT_OF_MEMORY;
    const csaw::WalkBatchLayout tl = csaw::walk_batch_layout(nreq, shape.walkers);
    std::vector<char> image(stt == CSAW_OK ? tl.bytes : 0);
    if (stt == CSAW_OK) csaw::walk_batch_image(reqs.data(), nreq, path_off.data(), image.data());
    if (stt == CSAW_OK && shape.walkers > 0 &&
        !x.to_device(x.dev + lay.o_starts, (const char*)starts.data(), (size_t)shape.walkers * sizeof(int32_t)))
        stt = CSAW_ERR_DEVICE;
    if (stt == CSAW_OK && !x.to_device(x.dev + lay.o_tab, image.data(), tl.bytes)) stt = CSAW_ERR_DEVICE;
    if (stt == CSAW_OK) {
        csaw_walk_args common{};
        common.bias_kind = batch[0]->bias;
        common.w_return = batch[0]->wr;
        common.w_common = batch[0]->wc;
        common.w_outward = batch[0]->wo;
        stt = csaw::walk_batch_in_scratch(g, &common, reqs.data(), nreq, (const int32_t*)(x.dev + lay.o_starts),
                                          (int32_t*)(x.dev + lay.o_paths), x.dev + lay.o_tab, steps.data(), x.st);
    }
    if (stt != CSAW_OK && nreq > 1) {  // isolate: every request on its own, so only a faulty one fails
        for (csaw_result* r : res) csaw_result_free(r);
        for (Request* r : batch) {
            std::vector<Request*> one{r};
            run_walk_batch(one, x, t0);
        }
        return;
    }
    bool direct = pool != nullptr;  // every request's paths in the pinned pool: copied straight there
    for (int32_t q = 0; q < nreq && direct; ++q) direct = res[q] && pool->owns(res[q]->paths);
    if (stt == CSAW_OK && path_off[nreq] > 0 && direct) {
        for (int32_t q = 0; q < nreq && stt == CSAW_OK; ++q)
            if (path_off[q + 1] > path_off[q] &&
                hipMemcpyAsync(res[q]->paths, x.dev + lay.o_paths + (size_t)path_off[q] * sizeof(int32_t),
                               (size_t)(path_off[q + 1] - path_off[q]) * sizeof(int32_t), hipMemcpyDeviceToHost,
                               x.st) != hipSuccess)
                stt = CSAW_ERR_DEVICE;
        if (stt == CSAW_OK && hipStreamSynchronize(x.st) != hipSuccess) stt = CSAW_ERR_DEVICE;
    } else if (stt == CSAW_OK && path_off[nreq] > 0) {
        // chunk [off, off + len) of the batch's paths goes to the requests it overlaps
        auto sink = [&](size_t off, const char* p, size_t len) {
            const int64_t e0 = (int64_t)(off / sizeof(int32_t)), e1 = e0 + (int64_t)(len / sizeof(int32_t));
            for (int32_t q = 0; q < nreq; ++q) {
                const int64_t s0 = std::max(e0, path_off[q]), s1 = std::min(e1, path_off[q + 1]);
                if (s0 >= s1) continue;
                std::memcpy(res[q]->paths + (s0 - path_off[q]), p + (s0 - e0) * sizeof(int32_t),
                            (size_t)(s1 - s0) * sizeof(int32_t));
            }
        };
        if (!x.to_host(x.dev + lay.o_paths, (size_t)path_off[nreq] * sizeof(int32_t), sink)) stt = CSAW_ERR_DEVICE;
    }
    const Clock::time_point t_end = Clock::now();
    for (int32_t q = 0; q < nreq; ++q) {
        if (res[q] && stt != CSAW_OK) {
            csaw_result_free(res[q]);
            res[q] = new_result(CSAW_REQUEST_WALK, stt);
        }
        if (res[q]) {
            res[q]->steps = stt == CSAW_OK ? steps[q] : 0;
            res[q]->queued_us = us_between(batch[q]->t_submit, t0);
            res[q]->total_us = us_between(batch[q]->t_submit, t_end);
        }
        finish(batch[q], res[q]);
    }
}

void csaw_server_s::run_sample_batch(std::vector<Request*>& batch, Exec& x, Clock::time_point t0) {
    const int32_t ni = (int32_t)batch.size();
    BatchShape shape;
    for (Request* r : batch) shape.add(*r);
    const int32_t L = shape.L;
    const BatchLayout lay = batch_layout(g, shape);
    csaw_status stt = lay.total <= x.bytes ? CSAW_OK : CSAW_ERR_OUT_OF_MEMORY;  // batches are formed to fit
    std::vector<int64_t> offs(ni + 1, 0);
    for (int32_t i = 0; i < ni; ++i) offs[i + 1] = offs[i] + (int64_t)batch[i]->seeds.size();
    std::vector<int32_t> fan((size_t)ni * std::max(L, 1), 0), bias(ni), seeds((size_t)offs[ni]);
    std::vector<uint64_t> ids(ni), keys(ni);
    for (int32_t i = 0; i < ni; ++i) {
        std::copy(batch[i]->fanouts.begin(), batch[i]->fanouts.end(), fan.begin() + (size_t)i * L);
        std::copy(batch[i]->seeds.begin(), batch[i]->seeds.end(), seeds.begin() + offs[i]);
        bias[i] = batch[i]->bias;
        ids[i] = batch[i]->id;
        keys[i] = batch[i]->rng_seed;
    }
    if (stt == CSAW_OK && offs[ni] > 0 &&
        !x.to_device(x.dev + lay.o_seeds, (const char*)seeds.data(), (size_t)offs[ni] * sizeof(int32_t)))
        stt = CSAW_ERR_DEVICE;
    csaw_sample_out out{};
    if (stt == CSAW_OK) {
        csaw_sample_args a{};
        a.num_instances = ni;
        a.seed_offsets = offs.data();
        a.seeds = (const int32_t*)(x.dev + lay.o_seeds);
        a.num_layers = L;
        a.fanouts = fan.data();
        a.fanout_stride = L;
        a.bias_kinds = bias.data();
        a.instance_ids = ids.data();
        a.rng_seeds = keys.data();
        out.src = (int32_t*)(x.dev + lay.o_src);
        out.dst = (int32_t*)(x.dev + lay.o_dst);
        out.edge_capacity = shape.edges;
        out.offsets = (int64_t*)(x.dev + lay.o_off);
        stt = csaw::sample_in_scratch(g, &a, &out, x.st, x.dev + lay.o_scratch, x.bytes - lay.o_scratch);
    }
    if (stt != CSAW_OK) {
        if (ni > 1) {  // isolate: every request on its own, so only a faulty one fails
            for (Request* r : batch) {
                std::vector<Request*> one{r};
                run_sample_batch(one, x, t0);
            }
            return;
        }
        csaw_result* res = new_result(CSAW_REQUEST_SAMPLE, stt);
        if (res) {
            res->batch_requests = 1;
            res->queued_us = us_between(batch[0]->t_submit, t0);
            res->total_us = us_between(batch[0]->t_submit, Clock::now());
        }
        return finish(batch[0], res);
    }
    const int64_t ne = out.num_edges;
    const size_t noff = (size_t)L * ni + 1;
    std::vector<int64_t> h_off(noff);
    bool ok = x.to_host(x.dev + lay.o_off, noff * sizeof(int64_t), [&h_off](size_t off, const char* p, size_t len) {
        std::memcpy((char*)h_off.data() + off, p, len);
    });
    // the segment offsets come from device memory: check them before they size
    // host copies (monotone, from 0 to ne <= capacity)
    ok = ok && ne >= 0 && ne <= shape.edges && h_off[0] == 0 && h_off[noff - 1] == ne;
    for (size_t j = 1; ok && j < noff; ++j) ok = h_off[j] >= h_off[j - 1];
    std::vector<csaw_result*> res(ni, nullptr);
    // the batch's result arrays as one run of the pool when it has room (one
    // copy fills them all), else one range or heap block each
    std::vector<size_t> sizes;
    std::vector<int64_t> cnts(ni, 0);
    for (int32_t i = 0; ok && i < ni; ++i) {
        for (int32_t l = 0; l < L; ++l) cnts[i] += h_off[(size_t)l * ni + i + 1] - h_off[(size_t)l * ni + i];
        sizes.push_back((size_t)std::max<int64_t>(cnts[i], 1) * sizeof(int32_t));  // src
        sizes.push_back(sizes.back());                                             // dst
    }
    std::vector<char*> run;
    if (!(ok && pool && pool->take_run(sizes, run))) run.clear();
    for (int32_t i = 0; ok && i < ni; ++i) {
        const int32_t Li = (int32_t)batch[i]->fanouts.size();
        res[i] = new_result(CSAW_REQUEST_SAMPLE, CSAW_OK);
        if (!res[i]) continue;
        res[i]->num_edges = cnts[i];
        res[i]->num_layers = Li;
        if (!run.empty()) {
            hold_pool(pool, res[i]);
            res[i]->src = (int32_t*)run[2 * i];
            res[i]->dst = (int32_t*)run[2 * i + 1];
        } else {
            res[i]->src = (int32_t*)result_array(pool, res[i], sizes[2 * i]);
            res[i]->dst = (int32_t*)result_array(pool, res[i], sizes[2 * i + 1]);
        }
        res[i]->layer_offsets = (int64_t*)std::malloc(((size_t)Li + 1) * sizeof(int64_t));
        if (!res[i]->src || !res[i]->dst || !res[i]->layer_offsets) {
            res[i]->status = CSAW_ERR_OUT_OF_MEMORY;
            continue;
        }
        int64_t w = 0;
        for (int32_t l = 0; l < Li; ++l) {
            res[i]->layer_offsets[l] = w;
            w += h_off[(size_t)l * ni + i + 1] - h_off[(size_t)l * ni + i];
        }
        res[i]->layer_offsets[Li] = w;
        // an instance has no edges in layers beyond its own
        for (int32_t l = Li; l < L; ++l)
            ok = ok && h_off[(size_t)l * ni + i + 1] == h_off[(size_t)l * ni + i];
    }
    // pieces of the run that no result took go back
    for (int32_t i = 0; i < ni && !run.empty(); ++i)
        if (!res[i] || res[i]->src != (int32_t*)run[2 * i]) {
            pool->give(run[2 * i]);
            pool->give(run[2 * i + 1]);
        }
    // segment (l, i) = edges [h_off[l*ni+i], h_off[l*ni+i+1]) go to instance i
    // at its layer-l offset; segments are in increasing edge order
    auto scatter = [&](int32_t* csaw_result::*field) {
        return [&, field](size_t off_bytes, const char* p, size_t len_bytes) {
            const int64_t e0 = (int64_t)(off_bytes / sizeof(int32_t)), e1 = e0 + (int64_t)(len_bytes / sizeof(int32_t));
            // first segment ending after e0
            size_t j = std::upper_bound(h_off.begin(), h_off.end(), e0) - h_off.begin();
            j = j > 0 ? j - 1 : 0;
            for (; j + 1 < noff && h_off[j] < e1; ++j) {
                const int64_t s0 = std::max(h_off[j], e0), s1 = std::min(h_off[j + 1], e1);
                if (s1 <= s0) continue;
                const int32_t l = (int32_t)(j / ni), i = (int32_t)(j % ni);
                csaw_result* r = res[i];
                if (!r || r->status != CSAW_OK) continue;
                const int64_t at = r->layer_offsets[l] + (s0 - h_off[j]);
                std::memcpy(r->*field + at, p + (s0 - e0) * sizeof(int32_t), (size_t)(s1 - s0) * sizeof(int32_t));
            }
        };
    };
    // the batch's arrays as one run of the pinned pool: a kernel lays the
    // edges out in the device block exactly as the run holds them (each
    // (layer, instance) segment at its request's layer offset), then one copy
    // moves the whole run (kernel stores into host memory over the bus ran at
    // 3 GB/s; the copy at 55 GB/s)
    const size_t nseg = noff - 1, tab_bytes = 2 * nseg * sizeof(int32_t*);
    const size_t span = run.empty() ? 0 : (size_t)(run.back() - run.front()) + sizes.back();
    bool direct = ok && !run.empty() && align_up(span) + tab_bytes <= lay.scratch;
    for (int32_t i = 0; direct && i < ni; ++i) direct = res[i] && res[i]->status == CSAW_OK;
    if (direct) {
        char* dspan = x.dev + lay.o_scratch;  // the call is done with its scratch
        char* dtab = dspan + align_up(span);
        std::vector<int32_t*> tab(2 * nseg, nullptr);
        for (size_t j = 0; j < nseg; ++j) {
            if (h_off[j + 1] == h_off[j]) continue;
            const csaw_result* r = res[j % ni];
            const int64_t at = r->layer_offsets[j / ni];
            tab[j] = (int32_t*)(dspan + ((const char*)(r->src + at) - run.front()));
            tab[nseg + j] = (int32_t*)(dspan + ((const char*)(r->dst + at) - run.front()));
        }
        ok = x.to_device(dtab, (const char*)tab.data(), tab_bytes);
        if (ok) {
            csaw::launch_scatter_segments((const int32_t*)(x.dev + lay.o_src), (const int32_t*)(x.dev + lay.o_dst),
                                          (const int64_t*)(x.dev + lay.o_off), (int64_t)nseg, ne,
                                          (int32_t* const*)dtab, (int32_t* const*)dtab + nseg, x.st);
            ok = hipGetLastError() == hipSuccess &&
                 hipMemcpyAsync(run.front(), dspan, span, hipMemcpyDeviceToHost, x.st) == hipSuccess &&
                 hipStreamSynchronize(x.st) == hipSuccess;
        }
    } else {
        ok = ok && x.to_host(x.dev + lay.o_src, (size_t)ne * sizeof(int32_t), scatter(&csaw_result::src)) &&
             x.to_host(x.dev + lay.o_dst, (size_t)ne * sizeof(int32_t), scatter(&csaw_result::dst));
    }
    const Clock::time_point t_end = Clock::now();
    for (int32_t i = 0; i < ni; ++i) {
        if (!ok) {
            csaw_result_free(res[i]);
            res[i] = new_result(CSAW_REQUEST_SAMPLE, CSAW_ERR_DEVICE);
        }
        if (res[i]) {
            res[i]->batch_requests = ni;
            res[i]->queued_us = us_between(batch[i]->t_submit, t0);
            res[i]->total_us = us_between(batch[i]->t_submit, t_end);
        }
        finish(batch[i], res[i]);
    }
}

void csaw_server_s::worker(Exec& x) {
    (void)hipSetDevice(device);
    for (;;) {
        std::vector<Request*> batch;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [this] { return !queue.empty() || stop; });
            if (queue.empty()) break;  // stop requested and drained
            Request* head = queue.front();
            queue.pop_front();
            batch.push_back(head);
            if (head->kind == CSAW_REQUEST_WALK) {
                // waiting walks of the same kind join while the batch's
                // device layout fits this executor's block and its walkers
                // stay within max_batch_walkers (smaller walk calls spread
                // the walks, and their copies to the host, over executors)
                WalkShape shape;
                shape.add(*head);
                for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < cfg.max_batch;) {
                    Request* r = *it;
                    if (r->kind == CSAW_REQUEST_WALK && same_walk_kind(*r, *head)) {
                        WalkShape with = shape;
                        with.add(*r);
                        if (with.walkers <= cfg.max_batch_walkers && walk_layout(with).total <= x.bytes) {
                            shape = with;
                            batch.push_back(r);
                            it = queue.erase(it);
                            continue;
                        }
                    }
                    ++it;
                }
            } else if (head->kind == CSAW_REQUEST_SAMPLE) {
                // continuous batching: every waiting sampling request that still
                // fits this executor's block joins, in arrival order
                BatchShape shape;
                shape.add(*head);
                for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < cfg.max_batch;) {
                    Request* r = *it;
                    if (r->kind == CSAW_REQUEST_SAMPLE) {
                        BatchShape with = shape;
                        with.add(*r);
                        if (batch_layout(g, with).total <= x.bytes) {
                            shape = with;
                            batch.push_back(r);
                            it = queue.erase(it);
                            continue;
                        }
                    }
                    ++it;
                }
            }
            for (Request* r : batch) state[r->ticket] = kRunning;
        }
        const Clock::time_point t0 = Clock::now();
        if (batch[0]->kind == CSAW_REQUEST_SAMPLE) run_sample_batch(batch, x, t0);
        else run_walk_batch(batch, x, t0);
        for (Request* r : batch) delete r;
    }
}

void csaw_server_s::free_execs() {
    for (Exec& x : execs) {
        if (x.st) (void)hipStreamSynchronize(x.st);
        for (int k = 0; k < 2; ++k) {
            if (x.ev[k]) (void)hipEventDestroy(x.ev[k]);
            if (x.stage[k]) (void)hipHostFree(x.stage[k]);
        }
        if (x.dev) (void)hipFree(x.dev);
        if (x.st) (void)hipStreamDestroy(x.st);
    }
    execs.clear();
    if (pool) pool->unref();  // results still holding ranges keep it alive
    pool = nullptr;
}

extern "C" {

csaw_status csaw_server_create(csaw_graph g, const csaw_server_config* cfg, csaw_server* out) {
    if (!g || !out) return CSAW_ERR_INVALID_ARG;
    *out = nullptr;
    csaw_server_config c{};
    if (cfg) c = *cfg;
    if (c.memory_budget_bytes < 0 || c.max_batch < 0 || c.queue_capacity < 0 || c.num_streams < 0 ||
        c.max_batch_walkers < 0 || c.result_pool_bytes < 0)
        return CSAW_ERR_INVALID_ARG;
    if (c.memory_budget_bytes == 0) c.memory_budget_bytes = int64_t(32) << 30;
    if (c.max_batch == 0) c.max_batch = 512;
    if (c.queue_capacity == 0) c.queue_capacity = 65536;
    if (c.num_streams == 0) c.num_streams = 2;
    if (c.max_batch_walkers == 0) c.max_batch_walkers = int64_t(1) << 18;
    if (c.num_streams > 16 || c.max_batch > (1 << 20)) return CSAW_ERR_INVALID_ARG;
    csaw_server s = new csaw_server_s();
    s->g = g;
    s->cfg = c;
    int64_t m = 0, max_deg = 0;
    int32_t sorted = 0;
    csaw_graph_info(g, &s->n, &m, &max_deg, &sorted);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return CSAW_ERR_DEVICE;
    }
    s->exec_bytes = (size_t)(c.memory_budget_bytes / c.num_streams) / kAlign * kAlign;
    s->execs.resize(c.num_streams);
    csaw_status st = CSAW_OK;
    if (c.result_pool_bytes > 0 && !(s->pool = HostPool::create((size_t)c.result_pool_bytes)))
        st = CSAW_ERR_OUT_OF_MEMORY;
    for (Exec& x : s->execs) {
        if (st != CSAW_OK) break;
        x.bytes = s->exec_bytes;
        if (hipStreamCreateWithFlags(&x.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&x.ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&x.ev[1], hipEventDisableTiming) != hipSuccess) {
            st = CSAW_ERR_DEVICE;
            break;
        }
        if (hipMalloc((void**)&x.dev, std::max<size_t>(x.bytes, kAlign)) != hipSuccess ||
            hipHostMalloc((void**)&x.stage[0], kStageBytes, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&x.stage[1], kStageBytes, hipHostMallocDefault) != hipSuccess) {
            st = CSAW_ERR_OUT_OF_MEMORY;
            break;
        }
    }
    // edge-weight and degree tables are built before serving, so that no
    // request builds them (and allocates) while others run
    if (st == CSAW_OK && !s->execs.empty()) {
        st = csaw::prepare_bias_tables(g, CSAW_BIAS_NEIGHBOR_DEGREE, s->execs[0].st);
        if (st == CSAW_OK) (void)csaw::prepare_bias_tables(g, CSAW_BIAS_EDGE_WEIGHT, s->execs[0].st);
    }
    if (st != CSAW_OK) {
        s->free_execs();
        delete s;
        return st;
    }
    for (Exec& x : s->execs) s->workers.emplace_back([s, &x] { s->worker(x); });
    *out = s;
    return CSAW_OK;
}

csaw_status csaw_server_submit(csaw_server s, const csaw_request* q, uint64_t* ticket) {
    if (!s || !q || !ticket) return CSAW_ERR_INVALID_ARG;
    Request* r = new Request();
    r->kind = q->kind;
    r->id = q->id;
    r->rng_seed = q->rng_seed;
    r->bias = q->bias_kind;
    if (q->kind == CSAW_REQUEST_SAMPLE) {
        if (q->num_seeds < 0 || (q->num_seeds > 0 && !q->seeds) || q->num_layers < 0 ||
            q->num_layers > CSAW_MAX_LAYERS || (q->num_layers > 0 && !q->fanouts) || q->bias_kind < 0 ||
            q->bias_kind > CSAW_BIAS_NEIGHBOR_DEGREE) {
            delete r;
            return CSAW_ERR_INVALID_ARG;
        }
        r->seeds.assign(q->seeds, q->seeds + q->num_seeds);
        r->fanouts.assign(q->fanouts, q->fanouts + q->num_layers);
        for (int32_t v : r->seeds)
            if (v < 0 || (int64_t)v >= s->n) {
                delete r;
                return CSAW_ERR_INVALID_ARG;
            }
        const int64_t offs[2] = {0, (int64_t)r->seeds.size()};
        csaw_sample_args a{};
        a.num_instances = 1;
        a.seed_offsets = offs;
        a.num_layers = q->num_layers;
        a.fanouts = r->fanouts.data();
        a.bias_kind = q->bias_kind;
        const csaw_status st = csaw::sample_plan_caps(s->g, &a, r->fcap, &r->max_edges);
        if (st != CSAW_OK) {
            delete r;
            return st;
        }
        BatchShape one;
        one.add(*r);
        r->need = batch_layout(s->g, one).total;
    } else if (q->kind == CSAW_REQUEST_WALK) {
        if (q->num_walkers < 0 || (q->num_walkers > 0 && !q->starts) || q->length < 0 || q->bias_kind < 0 ||
            q->bias_kind > CSAW_BIAS_METROPOLIS_HASTINGS) {
            delete r;
            return CSAW_ERR_INVALID_ARG;
        }
        r->starts.assign(q->starts, q->starts + q->num_walkers);
        for (int32_t v : r->starts)
            if (v < 0 || (int64_t)v >= s->n) {
                delete r;
                return CSAW_ERR_INVALID_ARG;
            }
        r->length = q->length;
        r->wr = q->w_return;
        r->wc = q->w_common;
        r->wo = q->w_outward;
        WalkShape one;
        one.add(*r);
        r->need = walk_layout(one).total;
    } else {
        delete r;
        return CSAW_ERR_INVALID_ARG;
    }
    if (r->need > s->exec_bytes) {  // not even alone in one executor's block
        delete r;
        return CSAW_ERR_OUT_OF_MEMORY;
    }
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int64_t)s->queue.size() >= s->cfg.queue_capacity || s->stop) {
            delete r;
            return CSAW_ERR_BUSY;
        }
        r->ticket = s->next_ticket++;
        s->state[r->ticket] = csaw_server_s::kQueued;
        *ticket = r->ticket;
        s->queue.push_back(r);
    }
    s->cv_work.notify_one();
    return CSAW_OK;
}

static csaw_status take_result(csaw_server s, uint64_t ticket, csaw_result** result) {
    auto it = s->done.find(ticket);
    if (it == s->done.end()) return CSAW_ERR_NOT_READY;
    *result = it->second;
    s->done.erase(it);
    s->state.erase(ticket);
    return *result ? CSAW_OK : CSAW_ERR_OUT_OF_MEMORY;
}

csaw_status csaw_server_poll(csaw_server s, uint64_t ticket, csaw_result** result) {
    if (!s || !result) return CSAW_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->state.count(ticket)) return CSAW_ERR_INVALID_ARG;
    return take_result(s, ticket, result);
}

csaw_status csaw_server_wait(csaw_server s, uint64_t ticket, int64_t timeout_us, csaw_result** result) {
    if (!s || !result) return CSAW_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->state.count(ticket)) return CSAW_ERR_INVALID_ARG;
    auto ready = [&] { return s->done.count(ticket) > 0; };
    if (timeout_us < 0) s->cv_done.wait(lk, ready);
    else s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    return take_result(s, ticket, result);
}

csaw_status csaw_server_cancel(csaw_server s, uint64_t ticket) {
    if (!s) return CSAW_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto st = s->state.find(ticket);
    if (st == s->state.end()) return CSAW_ERR_INVALID_ARG;
    if (st->second != csaw_server_s::kQueued) return CSAW_ERR_BUSY;  // running or done: too late
    auto it = std::find_if(s->queue.begin(), s->queue.end(), [ticket](Request* r) { return r->ticket == ticket; });
    if (it == s->queue.end()) return CSAW_ERR_BUSY;
    Request* r = *it;
    s->queue.erase(it);
    csaw_result* res = new_result(r->kind, CSAW_ERR_CANCELLED);
    if (res) res->queued_us = res->total_us = us_between(r->t_submit, Clock::now());
    s->done[ticket] = res;
    st->second = csaw_server_s::kDone;
    delete r;
    s->cv_done.notify_all();
    return CSAW_OK;
}

csaw_status csaw_server_memory(csaw_server s, int64_t* device_bytes, int64_t* pinned_host_bytes) {
    if (!s) return CSAW_ERR_INVALID_ARG;
    if (device_bytes) *device_bytes = (int64_t)(s->exec_bytes * s->execs.size());
    if (pinned_host_bytes) *pinned_host_bytes = (int64_t)(2 * kStageBytes * s->execs.size());
    return CSAW_OK;
}

void csaw_result_free(csaw_result* r) {
    if (!r) return;
    ResultBox* b = reinterpret_cast<ResultBox*>(r);
    for (void* p : {(void*)r->src, (void*)r->dst, (void*)r->layer_offsets, (void*)r->paths}) {
        if (b->pool && b->pool->owns(p)) b->pool->give(p);
        else std::free(p);
    }
    if (b->pool) b->pool->unref();
    delete b;
}

csaw_status csaw_server_destroy(csaw_server s) {
    if (!s) return CSAW_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& kv : s->done) csaw_result_free(kv.second);
    s->free_execs();
    delete s;
    return CSAW_OK;
}

}  // extern "C"
