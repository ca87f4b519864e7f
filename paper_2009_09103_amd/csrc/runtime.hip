// runtime.hip -- host runtime and C-ABI of libcsaw (declared in include/csaw.h).
//
// Graph residency, argument validation, capacity planning, per-call device
// workspaces, the per-layer launch sequence of neighbor sampling and the
// walk launch. Every step of the selection itself runs in the kernels of
// sample_kernels.hip / walk_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/csaw.h"
#include "internal.h"
#include "kernels.h"

using namespace csaw;

// Scratch memory of the entry point that allocates nothing (device frontier
// arrays, control block, tables and instance bitmaps of one sampling call).
// Host code never passes this name to a kernel: it passes the per-device
// address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[CSAW_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string t_err;

csaw_status fail(csaw_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return st;
}

#define HIP_OR_FAIL(expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            return fail(e_ == hipErrorOutOfMemory ? CSAW_ERR_OUT_OF_MEMORY : CSAW_ERR_DEVICE,   \
                        "%s failed: %s", #expr, hipGetErrorString(e_));                           \
        }                                                                                         \
    } while (0)

// ------------------------------------------------------------- profiling
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
std::atomic<bool> g_prof{false};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof_recs;

// Timing of a scope while profiling is on. A scope around one kernel hands
// its events to the launch (ev()), which fills them with the kernel's own
// start and stop; a scope around several launches records them on the stream.
struct ProfScope {
    const char* name;
    hipStream_t s;
    bool kernel;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(const char* n, hipStream_t st, bool one_kernel = false) : name(n), s(st), kernel(one_kernel) {
        if (!g_prof.load(std::memory_order_relaxed)) return;
        if (hipEventCreate(&a) != hipSuccess) {
            a = nullptr;
            return;
        }
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            a = b = nullptr;
            return;
        }
        if (!kernel) (void)hipEventRecord(a, s);
    }
    LaunchEvents ev() const {
        LaunchEvents e;
        if (kernel && a) {
            e.start = a;
            e.stop = b;
        }
        return e;
    }
    ~ProfScope() {
        if (!a) return;
        if (!kernel) (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_recs.push_back({name, a, b});
    }
};

// ------------------------------------------------------------ workspace
// Source of workspace device memory: the caller's allocator (csaw_set_allocator)
// or hipMalloc; each buffer keeps the pair it came from for its release.
struct DevAllocator {
    csaw_alloc_fn alloc = nullptr;
    csaw_free_fn release = nullptr;
    void* user = nullptr;
};
std::mutex g_alloc_mu;
DevAllocator g_alloc;

hipError_t dev_alloc(DevAllocator& from, void** p, size_t bytes) {
    DevAllocator a;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        a = g_alloc;
    }
    from = a;
    if (!a.alloc) return hipMalloc(p, bytes);
    *p = a.alloc(bytes, a.user);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_release(const DevAllocator& from, void* p) {
    if (!p) return;
    if (from.release) from.release(p, from.user);
    else (void)hipFree(p);
}

struct Workspace {
    DevAllocator arena_from, bitmaps_from;
    char* arena = nullptr;
    size_t arena_cap = 0;
    uint32_t* bitmaps = nullptr;  // visited | next, zero between calls
    size_t bitmap_words = 0;
    char* pinned = nullptr;        // fine-grained host memory: kernels read and write it directly
    char* pinned_dev = nullptr;    // its device address
    size_t pinned_cap = 0;
    // side stream for the long-list kernels, forked from and joined back into
    // the caller's stream with events (default priority)
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // captured launch sequences of csaw_sample, keyed by every value they bake in
    hipStream_t capture = nullptr;
    std::vector<std::pair<std::vector<int64_t>, hipGraphExec_t>> graphs;

    void drop_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
    hipGraphExec_t find_graph(const std::vector<int64_t>& key) const {
        for (auto& kv : graphs)
            if (kv.first == key) return kv.second;
        return nullptr;
    }
    void put_graph(const std::vector<int64_t>& key, hipGraphExec_t exec) {
        if (graphs.size() >= 8) {
            (void)hipGraphExecDestroy(graphs.front().second);
            graphs.erase(graphs.begin());
        }
        graphs.emplace_back(key, exec);
    }

    ~Workspace() {
        drop_graphs();
        if (capture) (void)hipStreamDestroy(capture);
        if (aux) (void)hipStreamDestroy(aux);
        if (join) (void)hipEventDestroy(join);
        if (fork) (void)hipEventDestroy(fork);
        dev_release(arena_from, arena);
        dev_release(bitmaps_from, bitmaps);
        if (pinned) (void)hipHostFree(pinned);
    }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device scratch of csaw_sample_noalloc: one array per device, resolved
// once per device with hipGetSymbolAddress; calls on a device are
// serialised, and each clears what must start at zero.
constexpr size_t kNoAllocScratchBytes = size_t(CSAW_NOALLOC_SCRATCH_BYTES);
constexpr size_t kWalkScratchBytes = kWalkScratch;  // step counter and bad-start flag of a walk call
constexpr int kMaxDevices = 64;
struct NoAllocDevice {
    std::mutex mu;
    bool ready = false;
    char* ptr = nullptr;  // device address of this device's scratch
};
NoAllocDevice g_noalloc[kMaxDevices];

// CSAW_GRAPH=0 in the environment turns off launch-sequence replay.
bool graphs_enabled() {
    static const bool on = [] {
        const char* e = std::getenv("CSAW_GRAPH");
        return !(e && e[0] == '0');
    }();
    return on;
}

struct Carver {
    size_t off = 0;
    template <class T>
    size_t take(size_t count) {
        const size_t at = off;
        off = align_up(off + count * sizeof(T), 256);
        return at;
    }
};

}  // namespace

struct csaw_graph_s {
    int64_t n = 0, m = 0, max_deg = 0;
    int device = 0;
    bool sorted = true;
    bool ew_streamed = false;  // edge weights exist but are streamed by partition (out-of-memory graph)
    void* rowptr_mem = nullptr;    // device row offsets (32- or 64-bit, see RowPtr)
    int32_t* dflag = nullptr;      // device word for checks over the whole graph
    int32_t symmetric = -1;        // every edge has its reverse (-1: not checked yet)
    RowPtr rowptr{nullptr, nullptr};
    int32_t* col = nullptr;
    uint32_t* ew = nullptr;
    uint32_t* degw = nullptr;
    int32_t* ppos_ew = nullptr;
    int32_t* ppos_deg = nullptr;
    uint64_t* gtab_ew = nullptr;   // chunk prefix tables of the long lists
    uint64_t* gtab_deg = nullptr;
    uint64_t* wtot_ew = nullptr;   // list totals per weight array
    uint64_t* wtot_deg = nullptr;
    uint64_t* ctab_ew = nullptr;   // running chunk totals of the long lists
    uint64_t* ctab_deg = nullptr;
    WalkEdge* wrec_ew = nullptr;   // walk guides: per-edge prefixes and neighbors,
    WalkEdge* wrec_deg = nullptr;  // per-vertex lists and totals, bucket brackets
    WalkVertex* wvtx_ew = nullptr;
    WalkVertex* wvtx_deg = nullptr;
    WalkBucket* wgd_ew = nullptr;
    WalkBucket* wgd_deg = nullptr;
    std::mutex mu;                       // lazy preparation + workspace pool
    std::vector<Workspace*> pool;
    std::atomic<int32_t> bound16{kDefaultBound16}, bound32{kDefaultBound32};  // sub-wave buckets
    std::atomic<int32_t> walk_guides{1};  // weighted walks build and use the walk guides

    GraphDev dev() const {
        GraphDev g;
        g.n = n;
        g.m = m;
        g.rowptr = rowptr;
        g.col = col;
        g.ew = ew;
        g.degw = degw;
        g.ppos_ew = ppos_ew;
        g.ppos_deg = ppos_deg;
        g.gtab_ew = gtab_ew;
        g.gtab_deg = gtab_deg;
        g.wtot_ew = wtot_ew;
        g.wtot_deg = wtot_deg;
        g.ctab_ew = ctab_ew;
        g.ctab_deg = ctab_deg;
        g.wrec_ew = wrec_ew;
        g.wrec_deg = wrec_deg;
        g.wvtx_ew = wvtx_ew;
        g.wvtx_deg = wvtx_deg;
        g.wgd_ew = wgd_ew;
        g.wgd_deg = wgd_deg;
        if (!walk_guides.load()) {  // walks and long-list draws take the chunk tables
            g.wrec_ew = g.wrec_deg = nullptr;
            g.wvtx_ew = g.wvtx_deg = nullptr;
            g.wgd_ew = g.wgd_deg = nullptr;
        }
        return g;
    }
};

namespace {

Workspace* acquire(csaw_graph g) {
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->pool.empty()) {
        Workspace* w = g->pool.back();
        g->pool.pop_back();
        return w;
    }
    return new Workspace();
}

void release(csaw_graph g, Workspace* w) {
    std::lock_guard<std::mutex> lk(g->mu);
    g->pool.push_back(w);
}

// A workspace borrowed for one call. If the call did not reach its end (a
// HIP error after work was enqueued), the stream is drained and the
// workspace dropped, since its bitmaps may no longer be all-zero.
struct Lease {
    csaw_graph g;
    Workspace* w;
    hipStream_t s;
    bool clean = false;
    ~Lease() {
        if (!w) return;  // a call without a workspace (device scratch)
        if (clean) {
            release(g, w);
        } else {
            (void)hipStreamSynchronize(s);
            delete w;
        }
    }
};

csaw_status ensure_arena(Workspace* w, size_t bytes) {
    if (w->arena_cap >= bytes) return CSAW_OK;
    w->drop_graphs();
    dev_release(w->arena_from, w->arena);  // no work uses it: every call drains its stream at its end
    w->arena = nullptr;
    w->arena_cap = 0;
    const size_t cap = std::max<size_t>(bytes + bytes / 4, 1 << 20);
    HIP_OR_FAIL(dev_alloc(w->arena_from, (void**)&w->arena, cap));
    w->arena_cap = cap;
    return CSAW_OK;
}

csaw_status ensure_pinned(Workspace* w, size_t bytes) {
    if (w->pinned_cap >= bytes) return CSAW_OK;
    w->drop_graphs();  // captured copies name the old staging buffer
    if (w->pinned) HIP_OR_FAIL(hipHostFree(w->pinned));
    w->pinned = nullptr;
    w->pinned_cap = 0;
    const size_t cap = std::max<size_t>(bytes + bytes / 4, 1 << 16);
    HIP_OR_FAIL(hipHostMalloc((void**)&w->pinned, cap, hipHostMallocCoherent | hipHostMallocMapped));
    HIP_OR_FAIL(hipHostGetDevicePointer((void**)&w->pinned_dev, w->pinned, 0));
    w->pinned_cap = cap;
    return CSAW_OK;
}

csaw_status ensure_streams(Workspace* w) {
    if (w->fork) return CSAW_OK;
    HIP_OR_FAIL(hipStreamCreateWithFlags(&w->aux, hipStreamNonBlocking));
    HIP_OR_FAIL(hipEventCreateWithFlags(&w->join, hipEventDisableTiming));
    HIP_OR_FAIL(hipEventCreateWithFlags(&w->fork, hipEventDisableTiming));
    HIP_OR_FAIL(hipStreamCreateWithFlags(&w->capture, hipStreamNonBlocking));
    return CSAW_OK;
}

csaw_status ensure_bitmaps(Workspace* w, size_t words, hipStream_t s) {
    if (w->bitmap_words >= words) return CSAW_OK;
    w->drop_graphs();
    dev_release(w->bitmaps_from, w->bitmaps);
    w->bitmaps = nullptr;
    w->bitmap_words = 0;
    HIP_OR_FAIL(dev_alloc(w->bitmaps_from, (void**)&w->bitmaps, words * sizeof(uint32_t)));
    launch_fill_u32(w->bitmaps, 0u, (int64_t)words, s);
    HIP_OR_FAIL(hipGetLastError());
    HIP_OR_FAIL(hipStreamSynchronize(s));
    w->bitmap_words = words;
    return CSAW_OK;
}

csaw_status prepare_bias(csaw_graph g, int32_t kind, hipStream_t s) {
    // a weight array's positive counts and chunk prefix table; ppos_* is set
    // last, once everything it stands for is on the device
    std::lock_guard<std::mutex> lk(g->mu);
    if (kind == kEdgeWeight && !g->ppos_ew) {
        if (!g->ew) return fail(CSAW_ERR_INVALID_ARG, "EDGE_WEIGHT bias needs edge weights");
        int32_t* pp = nullptr;
        if (!g->gtab_ew)
            HIP_OR_FAIL(hipMalloc((void**)&g->gtab_ew, (size_t)chunk_table_rows(g->m) * kChunkGroups * sizeof(uint64_t)));
        if (!g->wtot_ew) HIP_OR_FAIL(hipMalloc((void**)&g->wtot_ew, std::max<int64_t>(g->n, 1) * sizeof(uint64_t)));
        if (!g->ctab_ew) HIP_OR_FAIL(hipMalloc((void**)&g->ctab_ew, (size_t)chunk_table_rows(g->m) * sizeof(uint64_t)));
        HIP_OR_FAIL(hipMalloc((void**)&pp, std::max<int64_t>(g->n, 1) * sizeof(int32_t)));
        launch_positive_counts(g->rowptr, g->ew, g->n, pp, g->wtot_ew, s);
        launch_chunk_table(g->rowptr, g->ew, g->n, g->gtab_ew, g->ctab_ew, s);
        const hipError_t e = hipGetLastError() != hipSuccess ? hipErrorLaunchFailure : hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipFree(pp);
            return fail(CSAW_ERR_DEVICE, "preparing EDGE_WEIGHT tables: %s", hipGetErrorString(e));
        }
        g->ppos_ew = pp;
    }
    if (kind == kNeighborDegree && !g->ppos_deg) {
        int32_t* pp = nullptr;
        if (!g->degw) HIP_OR_FAIL(hipMalloc((void**)&g->degw, std::max<int64_t>(g->m, 1) * sizeof(uint32_t)));
        if (!g->gtab_deg)
            HIP_OR_FAIL(hipMalloc((void**)&g->gtab_deg, (size_t)chunk_table_rows(g->m) * kChunkGroups * sizeof(uint64_t)));
        if (!g->wtot_deg) HIP_OR_FAIL(hipMalloc((void**)&g->wtot_deg, std::max<int64_t>(g->n, 1) * sizeof(uint64_t)));
        if (!g->ctab_deg) HIP_OR_FAIL(hipMalloc((void**)&g->ctab_deg, (size_t)chunk_table_rows(g->m) * sizeof(uint64_t)));
        HIP_OR_FAIL(hipMalloc((void**)&pp, std::max<int64_t>(g->n, 1) * sizeof(int32_t)));
        launch_degree_weights(g->rowptr, g->col, g->m, g->degw, s);
        launch_positive_counts(g->rowptr, g->degw, g->n, pp, g->wtot_deg, s);
        launch_chunk_table(g->rowptr, g->degw, g->n, g->gtab_deg, g->ctab_deg, s);
        const hipError_t e = hipGetLastError() != hipSuccess ? hipErrorLaunchFailure : hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipFree(pp);
            return fail(CSAW_ERR_DEVICE, "preparing NEIGHBOR_DEGREE tables: %s", hipGetErrorString(e));
        }
        g->ppos_deg = pp;
    }
    return CSAW_OK;
}

// The walk guide tables of a weight array whose bias tables exist (per-edge
// prefix and neighbor records, 16 bytes per edge; per-vertex list records,
// 16 bytes per vertex, when m < 2^32; buckets, 16 bytes each and at most two
// per edge), built once; a graph without them walks through the chunk
// tables.
csaw_status prepare_walk_guides(csaw_graph g, int32_t kind, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g->mu);
    const bool dg = kind == kNeighborDegree;
    if (kind != kEdgeWeight && !dg) return CSAW_OK;
    if ((dg ? g->wgd_deg : g->wgd_ew) || g->m <= 0) return CSAW_OK;
    const uint32_t* w = dg ? g->degw : g->ew;
    const uint64_t* tot = dg ? g->wtot_deg : g->wtot_ew;
    if (!w || !tot || !(dg ? g->ppos_deg : g->ppos_ew)) return CSAW_OK;
    WalkEdge* rec = nullptr;
    WalkVertex* vtx = nullptr;
    WalkBucket* gd = nullptr;
    const bool small = g->m < (int64_t(1) << 32);  // vertex records hold 32-bit list offsets
    if (hipMalloc((void**)&rec, (size_t)g->m * sizeof(WalkEdge)) != hipSuccess ||
        (small && hipMalloc((void**)&vtx, (size_t)std::max<int64_t>(g->n, 1) * sizeof(WalkVertex)) != hipSuccess) ||
        hipMalloc((void**)&gd, (size_t)(kGuideBucketsPerEdge * g->m + g->n) * sizeof(WalkBucket)) != hipSuccess) {
        if (rec) (void)hipFree(rec);
        if (vtx) (void)hipFree(vtx);
        return fail(CSAW_ERR_OUT_OF_MEMORY, "walk guide tables: allocation failed");
    }
    launch_walk_guides(g->rowptr, g->col, w, tot, g->n, rec, vtx, gd, s);
    const hipError_t e = hipGetLastError() != hipSuccess ? hipErrorLaunchFailure : hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(rec);
        if (vtx) (void)hipFree(vtx);
        (void)hipFree(gd);
        return fail(CSAW_ERR_DEVICE, "building the walk guide tables: %s", hipGetErrorString(e));
    }
    (dg ? g->wrec_deg : g->wrec_ew) = rec;
    (dg ? g->wvtx_deg : g->wvtx_ew) = vtx;
    (dg ? g->wgd_deg : g->wgd_ew) = gd;
    return CSAW_OK;
}

int64_t sat_mul(int64_t a, int64_t b) {
    if (a == 0 || b == 0) return 0;
    if (a > INT64_MAX / b) return INT64_MAX;
    return a * b;
}
int64_t sat_add(int64_t a, int64_t b) { return (a > INT64_MAX - b) ? INT64_MAX : a + b; }

struct SamplePlan {
    int32_t ni = 0, L = 0;
    std::vector<int32_t> fan;       // [(L+1) * ni], effective, zero row appended
    std::vector<int32_t> bias;      // [ni]
    std::vector<int64_t> fcap;      // [L+1] frontier capacity per layer
    int64_t max_edges = 0;
    int64_t total_seeds = 0;
    bool uses_deg = false, uses_ew = false;
    int32_t rounds = kDefaultRounds;
};

csaw_status plan_sample(csaw_graph g, const csaw_sample_args* a, SamplePlan& P, bool need_seeds) {
    if (!g) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    if (!a) return fail(CSAW_ERR_INVALID_ARG, "args is NULL");
    if (a->num_instances < 0) return fail(CSAW_ERR_INVALID_ARG, "num_instances < 0");
    if (a->num_layers < 0 || a->num_layers > CSAW_MAX_LAYERS)
        return fail(CSAW_ERR_INVALID_ARG, "num_layers must be in [0, %d]", CSAW_MAX_LAYERS);
    const int32_t ni = a->num_instances, L = a->num_layers;
    P.ni = ni;
    P.L = L;
    if (ni > 0 && !a->seed_offsets) return fail(CSAW_ERR_INVALID_ARG, "seed_offsets is NULL");
    if (L > 0 && ni > 0 && !a->fanouts) return fail(CSAW_ERR_INVALID_ARG, "fanouts is NULL");
    if (a->fanout_stride != 0 && a->fanout_stride < L)
        return fail(CSAW_ERR_INVALID_ARG, "fanout_stride must be 0 or >= num_layers");
    if (a->rounds < CSAW_DIRECT_ONLY || a->rounds > CSAW_ROUNDS)
        return fail(CSAW_ERR_INVALID_ARG, "rounds must be CSAW_DIRECT_ONLY, 0 (default) or 1..%d", CSAW_ROUNDS);
    P.rounds = a->rounds == 0 ? kDefaultRounds : (a->rounds == CSAW_DIRECT_ONLY ? 0 : a->rounds);
    if (ni > 0) {
        if (a->seed_offsets[0] != 0) return fail(CSAW_ERR_INVALID_ARG, "seed_offsets[0] != 0");
        for (int32_t i = 0; i < ni; ++i)
            if (a->seed_offsets[i + 1] < a->seed_offsets[i])
                return fail(CSAW_ERR_INVALID_ARG, "seed_offsets decreases at %d", i);
        P.total_seeds = a->seed_offsets[ni];
        if (need_seeds && P.total_seeds > 0 && !a->seeds) return fail(CSAW_ERR_INVALID_ARG, "seeds is NULL");
    }
    P.bias.resize(ni);
    for (int32_t i = 0; i < ni; ++i) {
        const int32_t k = a->bias_kinds ? a->bias_kinds[i] : a->bias_kind;
        if (k != kUniform && k != kEdgeWeight && k != kNeighborDegree)
            return fail(CSAW_ERR_INVALID_ARG, "bias kind %d is not a sampling bias (instance %d)", k, i);
        if (k == kEdgeWeight && !g->ew && !g->ew_streamed)
            return fail(CSAW_ERR_INVALID_ARG, "EDGE_WEIGHT bias without edge weights");
        P.bias[i] = k;
        P.uses_deg |= (k == kNeighborDegree);
        P.uses_ew |= (k == kEdgeWeight);
    }
    P.fan.assign((size_t)(L + 1) * ni, 0);
    P.fcap.assign(L + 1, 0);
    std::vector<int64_t> B(ni);
    for (int32_t i = 0; i < ni; ++i) B[i] = std::min<int64_t>(a->seed_offsets[i + 1] - a->seed_offsets[i], g->n);
    for (int32_t i = 0; i < ni; ++i) P.fcap[0] = sat_add(P.fcap[0], B[i]);
    for (int32_t i = 0; i < ni; ++i) {
        const int32_t* row = a->fanouts + (a->fanout_stride ? (int64_t)i * a->fanout_stride : 0);
        bool stopped = false;
        for (int32_t l = 0; l < L; ++l) {
            const int32_t f = row[l];
            if (f < -1 || f > 0xFFFF) return fail(CSAW_ERR_INVALID_ARG, "fanout %d out of range", f);
            if (f == 0) stopped = true;
            P.fan[(size_t)l * ni + i] = stopped ? 0 : f;
        }
    }
    for (int32_t l = 0; l < L; ++l) {
        int64_t next_cap = 0;
        for (int32_t i = 0; i < ni; ++i) {
            const int32_t f = P.fan[(size_t)l * ni + i];
            if (f == 0) {
                B[i] = 0;
                continue;
            }
            const int64_t per = f < 0 ? g->max_deg : std::min<int64_t>(f, g->max_deg);
            const int64_t e = std::min<int64_t>(sat_mul(B[i], per), g->m);
            P.max_edges = sat_add(P.max_edges, e);
            B[i] = P.fan[(size_t)(l + 1) * ni + i] != 0 ? std::min<int64_t>(e, g->n) : 0;
            next_cap = sat_add(next_cap, B[i]);
        }
        P.fcap[l + 1] = next_cap;
    }
    return CSAW_OK;
}

int64_t bitmap_words_per_instance(int64_t n) { return (int64_t)align_up((size_t)((n + 31) / 32), 4); }
// summary words per instance of a sparse build: one bit per bitmap word
int64_t summary_words_per_instance(int64_t nwp) { return (int64_t)align_up((size_t)((nwp + 31) / 32), 4); }

// Device memory of one sampling call, from its shape alone: the arena (control
// block, look-back words, tables, per-entry arrays, frontiers), then, for calls
// in a caller's scratch, the two bitmaps and the copy of the final control
// block. The small tables have the same layout in host memory.
struct SampleLayout {
    bool sparse;                   // frontier builds through a summary bitmap and a dirty-word list
    int64_t nsw;                   // summary words per instance (sparse)
    int64_t bitmap_words;          // visited, next and (sparse) the summary
    size_t t_fan, t_bias, t_iid, t_key, t_soff, tab_bytes;
    size_t o_ctl, o_status, ctl_words, o_tab, o_cnt, o_off, o_fbeg, o_fdeg, o_fpos, o_bigs, o_dirty;
    std::vector<size_t> o_fv, o_fi;
    size_t arena;                  // bytes of the arena part
    size_t o_bits, o_copy, scratch;
    int64_t nb_build;
};

bool layout_sample(int32_t ni, int32_t L, const std::vector<int64_t>& fcap, int64_t nwp, SampleLayout& y) {
    int64_t maxF = 0, sumF = 0;
    for (int l = 0; l <= L; ++l) {
        maxF = std::max(maxF, fcap[l]);
        sumF = sat_add(sumF, fcap[l]);
    }
    if (sumF > (int64_t(1) << 40)) return false;
    const int64_t words = nwp * ni;
    y.sparse = words > kSparseWords;
    y.nsw = y.sparse ? summary_words_per_instance(nwp) : 0;
    y.bitmap_words = words * 2 + y.nsw * ni;
    if (y.sparse) {  // look-back words for the compaction and for the widest dirty-word build
        y.nb_build = dirty_compact_blocks(y.nsw * ni);
        for (int l = 0; l <= L; ++l) y.nb_build = std::max(y.nb_build, sparse_build_blocks(fcap[l]));
    } else {
        y.nb_build = frontier_build_blocks(words);
    }
    size_t tb = 0;
    y.t_fan = tb;
    tb += (size_t)(L + 1) * ni * sizeof(int32_t);
    y.t_bias = tb;
    tb += (size_t)ni * sizeof(int32_t);
    y.t_iid = tb;
    tb = align_up(tb + (size_t)ni * sizeof(uint32_t), 8);
    y.t_key = tb;
    tb += (size_t)ni * sizeof(uint64_t);
    y.t_soff = tb;
    tb += ((size_t)ni + 1) * sizeof(int64_t);
    y.tab_bytes = tb;
    Carver cv;
    // the control block and the look-back words are adjacent: one fill clears both
    y.o_ctl = cv.take<SampleCtl>(1);
    y.o_status = cv.take<unsigned long long>((size_t)y.nb_build * 4);
    y.ctl_words = (y.o_status - y.o_ctl) / 4 + (size_t)y.nb_build * 8;
    y.o_tab = cv.take<char>(y.tab_bytes);
    const size_t F = (size_t)std::max<int64_t>(maxF, 1);
    y.o_cnt = cv.take<int32_t>(F);
    y.o_off = cv.take<int64_t>(F);
    y.o_fbeg = cv.take<int64_t>(F);
    y.o_fdeg = cv.take<int32_t>(F);
    y.o_fpos = cv.take<int32_t>(F);
    y.o_bigs = cv.take<int32_t>(F);
    y.o_dirty = y.sparse ? cv.take<int64_t>(F) : 0;  // a dirty word holds at least one frontier vertex
    y.o_fv.assign(L + 1, 0);
    y.o_fi.assign(L + 1, 0);
    for (int l = 0; l <= L; ++l) {
        y.o_fv[l] = cv.take<int32_t>((size_t)std::max<int64_t>(fcap[l], 1));
        y.o_fi[l] = cv.take<int32_t>((size_t)std::max<int64_t>(fcap[l], 1));
    }
    y.arena = cv.off;
    y.o_bits = align_up(cv.off, 256);
    y.o_copy = align_up(y.o_bits + (size_t)y.bitmap_words * sizeof(uint32_t), 256);
    y.scratch = y.o_copy + sizeof(SampleCtl);
    return true;
}

// Host check of a CSR graph (O(n + m)): bounds, monotone offsets, ids in
// range; reports the longest list and whether every list is sorted.
// Device row offsets from the host's int64 array: 32-bit words when every
// offset fits (m < 2^32; half the bytes of each row read on the device),
// else 64-bit. *mem is the allocation, *rp the view kernels use. The
// narrowing goes through a host buffer that must outlive the copy, so the
// copy is waited for.
hipError_t upload_rowptr(int64_t n, int64_t m, const int64_t* host, void** mem, RowPtr* rp, hipStream_t s) {
    const bool narrow = m <= (int64_t)UINT32_MAX;
    const size_t bytes = (size_t)(n + 1) * (narrow ? sizeof(uint32_t) : sizeof(int64_t));
    hipError_t e = hipMalloc(mem, bytes);
    if (e != hipSuccess) return e;
    if (narrow) {
        std::vector<uint32_t> w32((size_t)n + 1);
        for (int64_t v = 0; v <= n; ++v) w32[(size_t)v] = (uint32_t)host[v];
        if ((e = hipMemcpyAsync(*mem, w32.data(), bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        *rp = RowPtr{(const uint32_t*)*mem, nullptr};
    } else {
        if ((e = hipMemcpyAsync(*mem, host, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        *rp = RowPtr{nullptr, (const int64_t*)*mem};
    }
    return hipSuccess;
}

csaw_status validate_csr(int64_t n, int64_t m, const int64_t* rowptr, const int32_t* col, int64_t* max_deg_out = nullptr,
                         bool* sorted_out = nullptr) {
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(CSAW_ERR_INVALID_ARG, "num_vertices out of range");
    if (m < 0 || m >= (int64_t(1) << 40)) return fail(CSAW_ERR_INVALID_ARG, "num_edges out of range");
    if (!rowptr) return fail(CSAW_ERR_INVALID_ARG, "rowptr is NULL");
    if (m > 0 && !col) return fail(CSAW_ERR_INVALID_ARG, "col is NULL");
    if (rowptr[0] != 0 || rowptr[n] != m) return fail(CSAW_ERR_INVALID_ARG, "rowptr must start at 0 and end at m");
    int64_t max_deg = 0;
    bool sorted = true;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t d = rowptr[v + 1] - rowptr[v];
        if (d < 0) return fail(CSAW_ERR_INVALID_ARG, "rowptr decreases at vertex %lld", (long long)v);
        max_deg = std::max(max_deg, d);
    }
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
            const int32_t x = col[e];
            if (x < 0 || (int64_t)x >= n) return fail(CSAW_ERR_INVALID_ARG, "col[%lld] = %d out of range", (long long)e, x);
            if (e > rowptr[v] && col[e - 1] > x) sorted = false;
        }
    }
    if (max_deg_out) *max_deg_out = max_deg;
    if (sorted_out) *sorted_out = sorted;
    return CSAW_OK;
}

}  // namespace

extern "C" {

const char* csaw_last_error(void) { return t_err.c_str(); }

const char* csaw_version(void) { return "libcsaw 0.1 (gfx950)"; }

csaw_status csaw_graph_create(int64_t n, int64_t m, const int64_t* rowptr, const int32_t* col,
                              const uint32_t* edge_weight, uint32_t flags, csaw_stream stream, csaw_graph* out) {
    t_err.clear();
    if (!out) return fail(CSAW_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (flags != 0) return fail(CSAW_ERR_INVALID_ARG, "flags must be 0");
    int64_t max_deg = 0;
    bool sorted = true;
    csaw_status vst = validate_csr(n, m, rowptr, col, &max_deg, &sorted);
    if (vst != CSAW_OK) return vst;
    hipStream_t s = (hipStream_t)stream;
    csaw_graph g = new csaw_graph_s();
    g->n = n;
    g->m = m;
    g->max_deg = max_deg;
    g->sorted = sorted;
    auto cleanup = [&](csaw_status st) {
        csaw_graph_destroy(g);
        return st;
    };
    if (hipGetDevice(&g->device) != hipSuccess) return cleanup(fail(CSAW_ERR_DEVICE, "hipGetDevice failed"));
    hipError_t e;
    if ((e = upload_rowptr(n, m, rowptr, &g->rowptr_mem, &g->rowptr, s)) != hipSuccess)
        return cleanup(fail(CSAW_ERR_OUT_OF_MEMORY, "row offsets: %s", hipGetErrorString(e)));
    if ((e = hipMalloc((void**)&g->dflag, 256)) != hipSuccess ||
        (e = hipMalloc((void**)&g->col, std::max<int64_t>(m, 1) * sizeof(int32_t))) != hipSuccess ||
        (edge_weight && (e = hipMalloc((void**)&g->ew, std::max<int64_t>(m, 1) * sizeof(uint32_t))) != hipSuccess))
        return cleanup(fail(CSAW_ERR_OUT_OF_MEMORY, "graph allocation failed: %s", hipGetErrorString(e)));
    if ((m > 0 && (e = hipMemcpyAsync(g->col, col, m * sizeof(int32_t), hipMemcpyHostToDevice, s)) != hipSuccess) ||
        (edge_weight && m > 0 &&
         (e = hipMemcpyAsync(g->ew, edge_weight, m * sizeof(uint32_t), hipMemcpyHostToDevice, s)) != hipSuccess) ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return cleanup(fail(CSAW_ERR_DEVICE, "graph upload failed: %s", hipGetErrorString(e)));
    if (edge_weight) {
        csaw_status st = prepare_bias(g, kEdgeWeight, s);
        if (st != CSAW_OK) return cleanup(st);
    }
    *out = g;
    return CSAW_OK;
}

csaw_status csaw_graph_destroy(csaw_graph g) {
    if (!g) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    for (Workspace* w : g->pool) delete w;
    if (g->rowptr_mem) (void)hipFree(g->rowptr_mem);
    if (g->dflag) (void)hipFree(g->dflag);
    if (g->col) (void)hipFree(g->col);
    if (g->ew) (void)hipFree(g->ew);
    if (g->degw) (void)hipFree(g->degw);
    if (g->ppos_ew) (void)hipFree(g->ppos_ew);
    if (g->ppos_deg) (void)hipFree(g->ppos_deg);
    if (g->gtab_ew) (void)hipFree(g->gtab_ew);
    if (g->gtab_deg) (void)hipFree(g->gtab_deg);
    if (g->wtot_ew) (void)hipFree(g->wtot_ew);
    if (g->wtot_deg) (void)hipFree(g->wtot_deg);
    if (g->ctab_ew) (void)hipFree(g->ctab_ew);
    if (g->ctab_deg) (void)hipFree(g->ctab_deg);
    for (void* q : {(void*)g->wrec_ew, (void*)g->wrec_deg, (void*)g->wvtx_ew, (void*)g->wvtx_deg, (void*)g->wgd_ew,
                    (void*)g->wgd_deg})
        if (q) (void)hipFree(q);
    delete g;
    return CSAW_OK;
}

csaw_status csaw_graph_info(csaw_graph g, int64_t* n, int64_t* m, int64_t* max_degree, int32_t* sorted) {
    if (!g) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (max_degree) *max_degree = g->max_deg;
    if (sorted) *sorted = g->sorted ? 1 : 0;
    return CSAW_OK;
}

csaw_status csaw_sample_bound(csaw_graph g, const csaw_sample_args* a, int64_t* max_edges) {
    t_err.clear();
    if (!max_edges) return fail(CSAW_ERR_INVALID_ARG, "max_edges is NULL");
    SamplePlan P;
    csaw_status st = plan_sample(g, a, P, false);
    if (st != CSAW_OK) return st;
    *max_edges = P.max_edges;
    return CSAW_OK;
}

// One sampling call. Device memory comes from a pooled workspace (tables
// staged through its pinned block, long lists on its side stream, the launch
// sequence captured and replayed), or, when scratch is set, from that
// device scratch only: tables copied in, every kernel on the caller's
// stream, launched directly, no allocation of any kind on the device.
struct Streamer;
static csaw_status stream_layer(Streamer& st, const SampleLayer& p, int32_t l, int64_t cap, bool big_path,
                                bool uses_ew, bool uses_deg, int32_t b16, int32_t b32, hipStream_t s);

static csaw_status sample_call(csaw_graph g, const csaw_sample_args* a, csaw_sample_out* out, csaw_stream stream,
                               char* scratch, size_t scratch_bytes, Streamer* streamer = nullptr) {
    if (!out) return fail(CSAW_ERR_INVALID_ARG, "out is NULL");
    SamplePlan P;
    csaw_status st = plan_sample(g, a, P, true);
    if (st != CSAW_OK) return st;
    if (out->edge_capacity < 0) return fail(CSAW_ERR_INVALID_ARG, "edge_capacity < 0");
    if (out->edge_capacity > 0 && (!out->src || !out->dst)) return fail(CSAW_ERR_INVALID_ARG, "src/dst is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_OR_FAIL(hipSetDevice(g->device));
    if (scratch) {
        // the bias tables are built (and allocated) on a bias kind's first use
        bool ready;
        {
            std::lock_guard<std::mutex> lk(g->mu);
            ready = (!P.uses_deg || g->ppos_deg) && (!P.uses_ew || g->ppos_ew);
        }
        if (!ready)
            return fail(CSAW_ERR_NOT_READY,
                        "the NEIGHBOR_DEGREE tables of this graph are not built yet: they are allocated by the first "
                        "csaw_sample or csaw_walk call with that bias");
    } else {
        if (P.uses_deg && (st = prepare_bias(g, kNeighborDegree, s)) != CSAW_OK) return st;
        if (P.uses_ew && (st = prepare_bias(g, kEdgeWeight, s)) != CSAW_OK) return st;
    }

    const int32_t ni = P.ni, L = P.L;
    const int32_t b16 = g->bound16.load(std::memory_order_relaxed), b32 = g->bound32.load(std::memory_order_relaxed);
    out->num_edges = 0;
    if (ni == 0) {
        if (out->offsets) HIP_OR_FAIL(hipMemsetAsync(out->offsets, 0, sizeof(int64_t), s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
        return CSAW_OK;
    }
    const int64_t nwp = bitmap_words_per_instance(g->n);
    const int64_t words = nwp * ni;
    SampleLayout lay;
    if (!layout_sample(ni, L, P.fcap, nwp, lay)) return fail(CSAW_ERR_OUT_OF_MEMORY, "frontier bound too large");
    const int64_t nb_build = lay.nb_build;
    const size_t t_fan = lay.t_fan, t_bias = lay.t_bias, t_iid = lay.t_iid, t_key = lay.t_key, t_soff = lay.t_soff;
    const size_t tab_bytes = lay.tab_bytes;
    const size_t o_ctl = lay.o_ctl, o_status = lay.o_status, ctl_words = lay.ctl_words, o_tab = lay.o_tab;
    const size_t o_cnt = lay.o_cnt, o_off = lay.o_off, o_fbeg = lay.o_fbeg, o_fdeg = lay.o_fdeg, o_fpos = lay.o_fpos,
                 o_bigs = lay.o_bigs;
    const std::vector<size_t>& o_fv = lay.o_fv;
    const std::vector<size_t>& o_fi = lay.o_fi;
    // weighted calls can have long-list entries (lists longer than kWaveMaxD,
    // or with a total weight of 2^32 or more)
    const bool big_path = P.uses_deg || P.uses_ew;
    const size_t o_hctl = align_up(tab_bytes, 64);
    Workspace* ws = nullptr;
    char* A = nullptr;
    uint32_t* bitmaps = nullptr;
    char* H = nullptr;                 // host image of the table block
    std::vector<char> host_tables;     // (device scratch calls)
    SampleCtl* ctl_copy = nullptr;     // where the final control block is copied (device address)
    if (scratch) {
        if (lay.scratch > scratch_bytes)
            return fail(CSAW_ERR_OUT_OF_MEMORY, "the call needs %zu bytes of device scratch, more than the %zu it has",
                        lay.scratch, scratch_bytes);
        A = scratch;
        bitmaps = (uint32_t*)(scratch + lay.o_bits);
        ctl_copy = (SampleCtl*)(scratch + lay.o_copy);
        host_tables.resize(o_hctl + sizeof(SampleCtl));
        H = host_tables.data();
    }
    Lease rel{g, nullptr, s};
    if (!scratch) {
        ws = acquire(g);
        rel.w = ws;
        if ((st = ensure_arena(ws, lay.arena)) != CSAW_OK) return st;
        if ((st = ensure_bitmaps(ws, (size_t)lay.bitmap_words, s)) != CSAW_OK) return st;
        if ((st = ensure_streams(ws)) != CSAW_OK) return st;
        if ((st = ensure_pinned(ws, o_hctl + sizeof(SampleCtl))) != CSAW_OK) return st;
        A = ws->arena;
        bitmaps = ws->bitmaps;
        H = ws->pinned;
        ctl_copy = (SampleCtl*)(ws->pinned_dev + o_hctl);
    }

    SampleCtl* ctl = (SampleCtl*)(A + o_ctl);
    int32_t* d_fan = (int32_t*)(A + o_tab + t_fan);
    int32_t* d_bias = (int32_t*)(A + o_tab + t_bias);
    int64_t* d_soff = (int64_t*)(A + o_tab + t_soff);
    unsigned long long* d_status = (unsigned long long*)(A + o_status);
    int32_t* d_cnt = (int32_t*)(A + o_cnt);
    int64_t* d_off = (int64_t*)(A + o_off);
    uint32_t* visited = bitmaps;
    uint32_t* next = bitmaps + words;
    uint32_t* summ = lay.sparse ? bitmaps + 2 * words : nullptr;

    // the small tables: one host block (pinned, read by the setup kernel; or
    // copied into the scratch)
    std::memcpy(H + t_fan, P.fan.data(), P.fan.size() * sizeof(int32_t));
    std::memcpy(H + t_bias, P.bias.data(), ni * sizeof(int32_t));
    uint32_t* h_iid = (uint32_t*)(H + t_iid);
    for (int32_t i = 0; i < ni; ++i)
        h_iid[i] = (uint32_t)(a->instance_ids ? a->instance_ids[i] : a->instance_base + (uint64_t)i);
    uint64_t* h_key = (uint64_t*)(H + t_key);
    for (int32_t i = 0; i < ni; ++i) h_key[i] = a->rng_seeds ? a->rng_seeds[i] : a->rng_seed;
    std::memcpy(H + t_soff, a->seed_offsets, ((size_t)ni + 1) * sizeof(int64_t));
    SampleCtl* h_ctl = (SampleCtl*)(H + o_hctl);
    // every device step of the call, enqueued on stream s
    auto enqueue = [&](hipStream_t s) -> csaw_status {
        // one kernel clears the control block and look-back words and copies
        // the table block straight from host memory (scratch calls copied it
        // before)
        if (scratch)
            launch_call_setup((uint32_t*)ctl, (int64_t)ctl_words, nullptr, nullptr, 0, s);
        else
            launch_call_setup((uint32_t*)ctl, (int64_t)ctl_words, (const uint32_t*)ws->pinned_dev,
                              (uint32_t*)(A + o_tab), (int64_t)(tab_bytes / 4), s);

        FrontierBuild fb;
        fb.g = g->dev();
        fb.next = next;
        fb.visited = visited;
        fb.nwords = words;
        fb.nwp = nwp;
        fb.nb = nb_build;
        fb.summ = summ;
        fb.nsw = lay.nsw;
        fb.dirty = lay.sparse ? (int64_t*)(A + lay.o_dirty) : nullptr;
        fb.nb_dirty = lay.sparse ? dirty_compact_blocks(lay.nsw * ni) : 0;
        fb.num_layers = L;
        fb.num_instances = ni;
        fb.bias = d_bias;
        fb.inst_id = (const uint32_t*)(A + o_tab + t_iid);
        fb.inst_key = (const uint64_t*)(A + o_tab + t_key);
        fb.burn = a->burn_threshold;
        fb.cnt = d_cnt;
        fb.off = d_off;
        fb.fbeg = (int64_t*)(A + o_fbeg);
        fb.fdeg = (int32_t*)(A + o_fdeg);
        fb.fpos = (int32_t*)(A + o_fpos);
        fb.bigs = (int32_t*)(A + o_bigs);
        fb.offsets = out->offsets;
        fb.ctl = ctl;
        fb.status = d_status;
        auto build = [&](int32_t l, LaunchEvents ev) {
            fb.layer = l;
            fb.fanout = d_fan + (size_t)l * ni;
            fb.fv = (int32_t*)(A + o_fv[l]);
            fb.fi = (int32_t*)(A + o_fi[l]);
            if (lay.sparse) fb.nb = sparse_build_blocks(P.fcap[l]);  // one thread per dirty word, at most one per entry
            launch_frontier_build(fb, s, ev);
        };
        {
            ProfScope ps("frontier_init", s);
            launch_mark_seeds(a->seeds, P.total_seeds, d_soff, ni, g->n, next, nwp, summ, lay.nsw, ctl, s);
            build(0, LaunchEvents{});
        }
        SampleLayer p;
        p.g = g->dev();
        p.num_instances = ni;
        p.inst_id = (const uint32_t*)(A + o_tab + t_iid);
        p.inst_key = (const uint64_t*)(A + o_tab + t_key);
        p.bias = d_bias;
        p.cnt = d_cnt;
        p.off = d_off;
        p.fbeg = (const int64_t*)(A + o_fbeg);
        p.fdeg = (const int32_t*)(A + o_fdeg);
        p.fpos = (const int32_t*)(A + o_fpos);
        p.bigs = (const int32_t*)(A + o_bigs);
        p.ctl = ctl;
        p.src = out->src;
        p.dst = out->dst;
        p.capacity = out->edge_capacity;
        p.visited = visited;
        p.next = next;
        p.nwp = nwp;
        p.summ = summ;
        p.nsw = lay.nsw;
        p.group16 = b16;
        p.group32 = b32;
        p.rounds = P.rounds;
        p.burn = a->burn_threshold;
        p.vlo = 0;  // every vertex (an out-of-memory schedule narrows it per partition)
        p.vhi = INT32_MAX;
        int computed_layers = 1;  // frontiers F_0 .. F_{computed_layers-1} exist
        for (int32_t l = 0; l < L; ++l) {
            p.layer = l;
            p.fanout = d_fan + (size_t)l * ni;
            p.fanout_next = d_fan + (size_t)(l + 1) * ni;
            p.fv = (const int32_t*)(A + o_fv[l]);
            p.fi = (const int32_t*)(A + o_fi[l]);
            const int64_t cap = P.fcap[l];
            if (streamer) {  // out of memory: partition by partition, each once resident
                if ((st = stream_layer(*streamer, p, l, cap, big_path, P.uses_ew, P.uses_deg, b16, b32, s)) != CSAW_OK)
                    return st;
                if (l + 1 < L && P.fcap[l + 1] > 0) {
                    build(l + 1, LaunchEvents{});
                    computed_layers = l + 2;
                }
                continue;
            }
            // the long-list path and the wavefront kernel touch disjoint outputs:
            // run them side by side (scratch calls: one after the other)
            hipStream_t aux = scratch ? s : ws->aux;
            if (!scratch) {
                HIP_OR_FAIL(hipEventRecord(ws->fork, s));
                HIP_OR_FAIL(hipStreamWaitEvent(aux, ws->fork, 0));
            }
            if (big_path) {
                ProfScope ps("select_big", aux, true);
                launch_select_big(p, (int)std::min<int64_t>(std::max<int64_t>((cap + 3) / 4, 1), 2048), aux,
                                  ps.ev());
            }
            if (b16 > 0 || b32 > 0) {
                ProfScope ps("select_small", s, true);
                // one wavefront per run of 64 entries, up to the resident slots
                const int grid = (int)std::min<int64_t>(std::max<int64_t>((cap + 255) / 256, 1), 2048);
                launch_select_small(p, grid, s, ps.ev());
            }
            {
                ProfScope ps("select_wave", s, true);
                // more wavefronts than resident slots (the dispatcher balances them),
                // each taking a short run of consecutive entries
                const int grid = (int)std::min<int64_t>(std::max<int64_t>((cap + 3) / 4, 1), 4096);
                launch_select(p, grid, s, ps.ev());
            }
            if (!scratch) {
                HIP_OR_FAIL(hipEventRecord(ws->join, aux));
                HIP_OR_FAIL(hipStreamWaitEvent(s, ws->join, 0));
            }
            if (l + 1 < L && P.fcap[l + 1] > 0) {
                ProfScope ps("frontier_build", s, true);
                build(l + 1, ps.ev());
                computed_layers = l + 2;
            }
        }
        {
            ProfScope ps("visited_clear", s, true);
            ClearVisited cl{};
            cl.num_layers = computed_layers;
            cl.fcount = ctl->fcount;
            cl.ctl = ctl;
            cl.host_ctl = ctl_copy;
            cl.visited = visited;
            cl.nwp = nwp;
            for (int l = 0; l < computed_layers; ++l) {
                cl.fv[l] = (const int32_t*)(A + o_fv[l]);
                cl.fi[l] = (const int32_t*)(A + o_fi[l]);
                cl.cap_entries = std::max(cl.cap_entries, P.fcap[l]);
            }
            launch_clear_visited(cl, s, ps.ev());
        }
        HIP_OR_FAIL(hipGetLastError());
        return CSAW_OK;
    };

    // the call's launch sequence, replayed from its captured graph when enabled
    if (streamer) {  // host decisions between layers: eager
        if ((st = enqueue(s)) != CSAW_OK) return st;
        HIP_OR_FAIL(hipStreamSynchronize(s));
    } else if (scratch) {
        // the tables, and zero bitmaps: the scratch keeps the last call's contents
        HIP_OR_FAIL(hipMemcpyAsync(A + o_tab, H, tab_bytes, hipMemcpyHostToDevice, s));
        launch_fill_u32(bitmaps, 0u, lay.bitmap_words, s);
        if ((st = enqueue(s)) != CSAW_OK) return st;
        HIP_OR_FAIL(hipMemcpyAsync(h_ctl, ctl, sizeof(SampleCtl), hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
    } else {
        if (graphs_enabled() && !g_prof.load(std::memory_order_relaxed)) {
            std::vector<int64_t> key = {ni, L, words, nwp, P.total_seeds, out->edge_capacity, (int64_t)(intptr_t)a->seeds,
                                        (int64_t)(intptr_t)out->src, (int64_t)(intptr_t)out->dst,
                                        (int64_t)(intptr_t)out->offsets, (int64_t)(intptr_t)ws->arena,
                                        (int64_t)(intptr_t)ws->bitmaps, (int64_t)(intptr_t)ws->pinned,
                                        (int64_t)big_path, b16, b32, P.rounds, (int64_t)a->burn_threshold};
            key.insert(key.end(), P.fcap.begin(), P.fcap.end());
            // the graph's arrays are baked into the kernel arguments too; the
            // bias tables of a weight array appear on its first use, so a
            // sequence captured before then must not serve a later call
            const GraphDev gd = g->dev();
            for (const void* q : {gd.rowptr.data(), (const void*)gd.col, (const void*)gd.ew, (const void*)gd.degw,
                                  (const void*)gd.ppos_ew, (const void*)gd.ppos_deg, (const void*)gd.gtab_ew,
                                  (const void*)gd.gtab_deg, (const void*)gd.wtot_ew, (const void*)gd.wtot_deg,
                                  (const void*)gd.ctab_ew, (const void*)gd.ctab_deg, (const void*)gd.wrec_ew,
                                  (const void*)gd.wrec_deg, (const void*)gd.wvtx_ew, (const void*)gd.wvtx_deg,
                                  (const void*)gd.wgd_ew, (const void*)gd.wgd_deg})
                key.push_back((int64_t)(intptr_t)q);
            key.push_back((int64_t)P.uses_deg);
            key.push_back((int64_t)P.uses_ew);
            hipGraphExec_t exec = ws->find_graph(key);
            if (!exec) {
                HIP_OR_FAIL(hipStreamBeginCapture(ws->capture, hipStreamCaptureModeRelaxed));
                const csaw_status cst = enqueue(ws->capture);
                hipGraph_t graph = nullptr;
                const hipError_t e = hipStreamEndCapture(ws->capture, &graph);
                if (cst != CSAW_OK) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return cst;
                }
                if (e != hipSuccess) return fail(CSAW_ERR_DEVICE, "capture failed: %s", hipGetErrorString(e));
                const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e2 != hipSuccess) return fail(CSAW_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e2));
                ws->put_graph(key, exec);
            }
            HIP_OR_FAIL(hipGraphLaunch(exec, s));
        } else {
            if ((st = enqueue(s)) != CSAW_OK) return st;
        }
        HIP_OR_FAIL(hipStreamSynchronize(s));
    }
    // a frontier build that gave up its look-back wrote entries at unknown
    // positions, so the bitmaps may not be clean: the workspace is dropped
    // (Lease) instead of going back to the pool
    if (h_ctl->lookback_stuck) return fail(CSAW_ERR_DEVICE, "frontier build did not complete its block chain");
    rel.clean = true;
    out->num_edges = L > 0 ? h_ctl->out_base[L] : 0;
    if (out->num_edges < 0) return fail(CSAW_ERR_DEVICE, "the device reported a negative edge count");
    if (h_ctl->bad_seed) return fail(CSAW_ERR_INVALID_ARG, "a seed is outside [0, n)");
    if (h_ctl->unsupported)
        return fail(CSAW_ERR_UNSUPPORTED, "a drawn fanout exceeds %d", CSAW_MAX_FANOUT);
    if (h_ctl->overflow || out->num_edges > out->edge_capacity)
        return fail(CSAW_ERR_OUT_OF_MEMORY, "edge_capacity %lld < %lld edges", (long long)out->edge_capacity,
                    (long long)out->num_edges);
    return CSAW_OK;
}

csaw_status csaw_sample(csaw_graph g, const csaw_sample_args* a, csaw_sample_out* out, csaw_stream stream) {
    t_err.clear();
    return sample_call(g, a, out, stream, nullptr, 0);
}

csaw_status csaw_sample_noalloc(csaw_graph g, const csaw_sample_args* a, csaw_sample_out* out, csaw_stream stream) {
    t_err.clear();
    if (!g) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    if (g->device < 0 || g->device >= kMaxDevices) return fail(CSAW_ERR_UNSUPPORTED, "device %d", g->device);
    HIP_OR_FAIL(hipSetDevice(g->device));
    NoAllocDevice& nd = g_noalloc[g->device];
    std::lock_guard<std::mutex> lk(nd.mu);
    if (!nd.ready) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CSAW_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        nd.ptr = (char*)p;
        nd.ready = true;
    }
    const csaw_status st = sample_call(g, a, out, stream, nd.ptr, kNoAllocScratchBytes);
    // an early error may leave work of this call in flight: it ends before
    // the next call may use the scratch
    if (st != CSAW_OK) (void)hipStreamSynchronize((hipStream_t)stream);
    return st;
}

}  // extern "C"

// ---------------------------------------------------------- out of memory
// A graph whose adjacency and weights stay in pinned host memory and reach
// the device one vertex-range partition at a time (Section V): the row
// offsets and per-vertex tables (positive counts, list totals) are resident,
// and so are the calls' frontiers and bitmaps; a partition's column ids,
// weights and chunk prefix rows are loaded into one of max_resident device
// slots when a layer has frontier entries in it. Partitions of a layer are
// taken busiest first (most edges to sample), those already resident before
// the others, and the next partition's transfer (copy stream) overlaps the
// current one's selection. The selection kernels see the slot through base
// pointers shifted by the partition's first edge and row, and take only the
// frontier entries of the partition's vertices, so every edge is the one the
// in-memory call writes at the same place.
struct csaw_pgraph_s {
    csaw_graph g = nullptr;       // resident part (no column ids or weights)
    int32_t np = 0;
    std::vector<int64_t> vb, eb;  // [np + 1] vertex and edge bounds of the partitions
    int64_t* d_vb = nullptr;
    bool has_ew = false;
    int32_t* h_col = nullptr;     // pinned host copies of the partitioned arrays
    uint32_t* h_ew = nullptr;
    uint32_t* h_degw = nullptr;
    uint64_t* h_gtab_ew = nullptr;
    uint64_t* h_gtab_deg = nullptr;
    struct Slot {
        int32_t part = -1;
        bool col = false, ew = false, degw = false;  // arrays of `part` present
        int64_t last_use = 0;
        char* mem = nullptr;
        int32_t* d_col = nullptr;
        uint32_t* d_ew = nullptr;
        uint32_t* d_degw = nullptr;
        uint64_t* d_gtab_ew = nullptr;
        uint64_t* d_gtab_deg = nullptr;
        hipEvent_t ready = nullptr, idle = nullptr;
    };
    std::vector<Slot> slots;
    int64_t slot_edges = 0, slot_rows = 0;
    hipStream_t copy = nullptr;
    unsigned long long* d_work = nullptr;  // [2 * np]
    unsigned long long* h_work = nullptr;  // pinned
    int64_t tick = 0;
    std::mutex mu;                         // one call at a time
    int64_t rows(int32_t q) const { return (eb[q + 1] >> kTabShift) - (eb[q] >> kTabShift); }
};

struct Streamer {
    csaw_pgraph pg;
    csaw_stream_stats* stats;
};

namespace {

// Loads the arrays of partition q that the call needs into slot x, on the
// copy stream, after the slot's last selection; the compute stream waits.
csaw_status load_partition(csaw_pgraph pg, csaw_pgraph_s::Slot& x, int32_t q, bool need_ew, bool need_deg,
                           hipStream_t s, csaw_stream_stats* stats) {
    if (x.part != q) {
        x.part = q;
        x.col = x.ew = x.degw = false;
    }
    const bool want_ew = need_ew && !x.ew, want_deg = need_deg && !x.degw;
    if (x.col && !want_ew && !want_deg) {
        HIP_OR_FAIL(hipStreamWaitEvent(s, x.ready, 0));  // a load still in flight from earlier
        return CSAW_OK;
    }
    const int64_t e0 = pg->eb[q], ne = pg->eb[q + 1] - e0;
    const int64_t r0 = pg->eb[q] >> kTabShift, nr = pg->rows(q);
    HIP_OR_FAIL(hipStreamWaitEvent(pg->copy, x.idle, 0));
    int64_t bytes = 0;
    auto up = [&](void* d, const void* h, size_t n) -> hipError_t {
        bytes += (int64_t)n;
        return n ? hipMemcpyAsync(d, h, n, hipMemcpyHostToDevice, pg->copy) : hipSuccess;
    };
    if (!x.col) HIP_OR_FAIL(up(x.d_col, pg->h_col + e0, (size_t)ne * 4));
    if (want_ew) {
        HIP_OR_FAIL(up(x.d_ew, pg->h_ew + e0, (size_t)ne * 4));
        HIP_OR_FAIL(up(x.d_gtab_ew, pg->h_gtab_ew + r0 * kChunkGroups, (size_t)nr * kChunkGroups * 8));
    }
    if (want_deg) {
        HIP_OR_FAIL(up(x.d_degw, pg->h_degw + e0, (size_t)ne * 4));
        HIP_OR_FAIL(up(x.d_gtab_deg, pg->h_gtab_deg + r0 * kChunkGroups, (size_t)nr * kChunkGroups * 8));
    }
    HIP_OR_FAIL(hipEventRecord(x.ready, pg->copy));
    HIP_OR_FAIL(hipStreamWaitEvent(s, x.ready, 0));
    x.col = true;
    x.ew |= want_ew;
    x.degw |= want_deg;
    if (stats) {
        stats->partition_loads += 1;
        stats->bytes_loaded += bytes;
    }
    return CSAW_OK;
}

}  // namespace

static csaw_status stream_layer(Streamer& st, const SampleLayer& p, int32_t l, int64_t cap, bool big_path,
                                bool uses_ew, bool uses_deg, int32_t b16, int32_t b32, hipStream_t s) {
    csaw_pgraph pg = st.pg;
    const int32_t np = pg->np;
    // the layer's work per partition
    HIP_OR_FAIL(hipMemsetAsync(pg->d_work, 0, (size_t)np * 2 * sizeof(unsigned long long), s));
    launch_partition_work(p.fv, p.cnt, p.ctl, l, std::max<int64_t>(cap, 1), pg->d_vb, np, pg->d_work, s);
    HIP_OR_FAIL(hipMemcpyAsync(pg->h_work, pg->d_work, (size_t)np * 2 * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    std::vector<int32_t> order;
    for (int32_t q = 0; q < np; ++q)
        if (pg->h_work[2 * q + 1] > 0) order.push_back(q);  // partitions with edges to sample
    auto slot_of = [&](int32_t q) -> int {
        for (size_t k = 0; k < pg->slots.size(); ++k)
            if (pg->slots[k].part == q) return (int)k;
        return -1;
    };
    // resident partitions first, then busiest first
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const bool ra = slot_of(a) >= 0, rb = slot_of(b) >= 0;
        if (ra != rb) return ra;
        return pg->h_work[2 * a + 1] > pg->h_work[2 * b + 1];
    });
    for (size_t i = 0; i < order.size(); ++i) {
        const int32_t q = order[i];
        int k = slot_of(q);
        if (k < 0) {  // a slot whose partition this layer no longer needs, least recently used
            auto needed_later = [&](int32_t part) {
                return std::find(order.begin() + i, order.end(), part) != order.end();
            };
            for (size_t c = 0; c < pg->slots.size(); ++c) {
                const auto& x = pg->slots[c];
                const bool free_c = x.part < 0 || !needed_later(x.part);
                const bool free_k = k >= 0 && (pg->slots[k].part < 0 || !needed_later(pg->slots[k].part));
                if (k < 0 || (free_c && !free_k) || (free_c == free_k && x.last_use < pg->slots[k].last_use))
                    k = (int)c;
            }
        }
        csaw_pgraph_s::Slot& x = pg->slots[k];
        csaw_status ls = load_partition(pg, x, q, uses_ew, uses_deg, s, st.stats);
        if (ls != CSAW_OK) return ls;
        x.last_use = ++pg->tick;
        SampleLayer pp = p;
        const int64_t e0 = pg->eb[q], r0 = pg->eb[q] >> kTabShift;
        pp.g.col = x.d_col - e0;  // indexed by global edge ids of the partition's lists
        pp.g.ew = x.d_ew ? x.d_ew - e0 : nullptr;
        pp.g.degw = x.d_degw ? x.d_degw - e0 : nullptr;
        pp.g.gtab_ew = x.d_gtab_ew ? x.d_gtab_ew - r0 * kChunkGroups : nullptr;
        pp.g.gtab_deg = x.d_gtab_deg ? x.d_gtab_deg - r0 * kChunkGroups : nullptr;
        pp.g.wrec_ew = pp.g.wrec_deg = nullptr;  // streamed lists have no walk guide
        pp.g.wvtx_ew = pp.g.wvtx_deg = nullptr;
        pp.g.wgd_ew = pp.g.wgd_deg = nullptr;
        pp.vlo = (int32_t)pg->vb[q];
        pp.vhi = (int32_t)std::min<int64_t>(pg->vb[q + 1], INT32_MAX);
        if (big_path) launch_select_big(pp, (int)std::min<int64_t>(std::max<int64_t>((cap + 3) / 4, 1), 2048), s);
        if (b16 > 0 || b32 > 0)
            launch_select_small(pp, (int)std::min<int64_t>(std::max<int64_t>((cap + 255) / 256, 1), 2048), s);
        launch_select(pp, (int)std::min<int64_t>(std::max<int64_t>((cap + 3) / 4, 1), 4096), s);
        HIP_OR_FAIL(hipGetLastError());
        HIP_OR_FAIL(hipEventRecord(x.idle, s));  // the slot may be reloaded after this
    }
    return CSAW_OK;
}

extern "C" {

csaw_status csaw_pgraph_destroy(csaw_pgraph pg) {
    if (!pg) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    if (pg->copy) (void)hipStreamSynchronize(pg->copy);
    for (auto& x : pg->slots) {
        if (x.ready) (void)hipEventSynchronize(x.ready);
        if (x.idle) (void)hipEventSynchronize(x.idle);
        if (x.ready) (void)hipEventDestroy(x.ready);
        if (x.idle) (void)hipEventDestroy(x.idle);
        if (x.mem) (void)hipFree(x.mem);
    }
    if (pg->copy) (void)hipStreamDestroy(pg->copy);
    if (pg->d_vb) (void)hipFree(pg->d_vb);
    if (pg->d_work) (void)hipFree(pg->d_work);
    if (pg->h_work) (void)hipHostFree(pg->h_work);
    for (void* h : {(void*)pg->h_col, (void*)pg->h_ew, (void*)pg->h_degw, (void*)pg->h_gtab_ew, (void*)pg->h_gtab_deg})
        if (h) (void)hipHostFree(h);
    if (pg->g) csaw_graph_destroy(pg->g);
    delete pg;
    return CSAW_OK;
}

csaw_status csaw_pgraph_create(int64_t n, int64_t m, const int64_t* rowptr, const int32_t* col,
                               const uint32_t* edge_weight, int32_t num_partitions, int32_t max_resident,
                               csaw_stream stream, csaw_pgraph* out) {
    t_err.clear();
    if (!out) return fail(CSAW_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (num_partitions < 1 || num_partitions > kMaxPartitionsHost)
        return fail(CSAW_ERR_INVALID_ARG, "num_partitions must be in [1, %d]", kMaxPartitionsHost);
    if (max_resident < 1 || max_resident > num_partitions)
        return fail(CSAW_ERR_INVALID_ARG, "max_resident must be in [1, num_partitions]");
    csaw_status st = validate_csr(n, m, rowptr, col);
    if (st != CSAW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    csaw_pgraph pg = new csaw_pgraph_s();
    auto cleanup = [&](csaw_status e) {
        csaw_pgraph_destroy(pg);
        return e;
    };
    csaw_graph g = new csaw_graph_s();
    pg->g = g;
    g->n = n;
    g->m = m;
    pg->has_ew = edge_weight != nullptr;
    g->ew_streamed = pg->has_ew;
    for (int64_t v = 0; v < n; ++v) g->max_deg = std::max(g->max_deg, rowptr[v + 1] - rowptr[v]);
    g->sorted = false;  // walks need sorted resident lists; this graph is for sampling
    if (hipGetDevice(&g->device) != hipSuccess) return cleanup(fail(CSAW_ERR_DEVICE, "hipGetDevice failed"));
    // partitions of about m / np edges each (whole lists)
    const int32_t np = num_partitions;
    pg->np = np;
    pg->vb.assign(np + 1, 0);
    pg->eb.assign(np + 1, 0);
    for (int32_t q = 1; q < np; ++q) {
        const int64_t target = (int64_t)((__int128)m * q / np);
        const int64_t v = std::lower_bound(rowptr, rowptr + n + 1, target) - rowptr;
        pg->vb[q] = std::max(pg->vb[q - 1], std::min<int64_t>(v, n));
    }
    pg->vb[np] = n;
    for (int32_t q = 0; q <= np; ++q) pg->eb[q] = rowptr[pg->vb[q]];
    for (int32_t q = 0; q < np; ++q) {
        pg->slot_edges = std::max(pg->slot_edges, pg->eb[q + 1] - pg->eb[q]);
        pg->slot_rows = std::max(pg->slot_rows, pg->rows(q));
    }
    const int64_t nv = std::max<int64_t>(n, 1);
    hipError_t e;
    if ((e = upload_rowptr(n, m, rowptr, &g->rowptr_mem, &g->rowptr, s)) != hipSuccess)
        return cleanup(fail(CSAW_ERR_OUT_OF_MEMORY, "row offsets: %s", hipGetErrorString(e)));
    if ((e = hipMalloc((void**)&g->ppos_deg, nv * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void**)&g->wtot_deg, nv * sizeof(uint64_t))) != hipSuccess ||
        (pg->has_ew && (e = hipMalloc((void**)&g->ppos_ew, nv * sizeof(int32_t))) != hipSuccess) ||
        (pg->has_ew && (e = hipMalloc((void**)&g->wtot_ew, nv * sizeof(uint64_t))) != hipSuccess) ||
        (e = hipMalloc((void**)&pg->d_vb, (np + 1) * sizeof(int64_t))) != hipSuccess ||
        (e = hipMalloc((void**)&pg->d_work, 2 * np * sizeof(unsigned long long))) != hipSuccess ||
        (e = hipHostMalloc((void**)&pg->h_work, 2 * np * sizeof(unsigned long long), hipHostMallocDefault)) !=
            hipSuccess)
        return cleanup(fail(CSAW_ERR_OUT_OF_MEMORY, "allocation failed: %s", hipGetErrorString(e)));
    // pinned host copies of the partitioned arrays
    const size_t me = (size_t)std::max<int64_t>(m, 1);
    const size_t trows = (size_t)chunk_table_rows(m) * kChunkGroups;
    if ((e = hipHostMalloc((void**)&pg->h_col, me * 4, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&pg->h_degw, me * 4, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&pg->h_gtab_deg, trows * 8, hipHostMallocDefault)) != hipSuccess ||
        (pg->has_ew && (e = hipHostMalloc((void**)&pg->h_ew, me * 4, hipHostMallocDefault)) != hipSuccess) ||
        (pg->has_ew && (e = hipHostMalloc((void**)&pg->h_gtab_ew, trows * 8, hipHostMallocDefault)) != hipSuccess))
        return cleanup(fail(CSAW_ERR_OUT_OF_MEMORY, "pinned host allocation failed: %s", hipGetErrorString(e)));
    if (m > 0) std::memcpy(pg->h_col, col, (size_t)m * 4);
    if (pg->has_ew && m > 0) std::memcpy(pg->h_ew, edge_weight, (size_t)m * 4);
    // device slots
    const size_t se = (size_t)std::max<int64_t>(pg->slot_edges, 1), sr = (size_t)std::max<int64_t>(pg->slot_rows, 1);
    pg->slots.resize(max_resident);
    if ((e = hipStreamCreateWithFlags(&pg->copy, hipStreamNonBlocking)) != hipSuccess)
        return cleanup(fail(CSAW_ERR_DEVICE, "stream: %s", hipGetErrorString(e)));
    for (auto& x : pg->slots) {
        Carver cv;
        const size_t o_col = cv.take<int32_t>(se), o_degw = cv.take<uint32_t>(se),
                     o_gdeg = cv.take<uint64_t>(sr * kChunkGroups);
        const size_t o_ew = pg->has_ew ? cv.take<uint32_t>(se) : 0,
                     o_gew = pg->has_ew ? cv.take<uint64_t>(sr * kChunkGroups) : 0;
        if ((e = hipMalloc((void**)&x.mem, cv.off)) != hipSuccess)
            return cleanup(fail(CSAW_ERR_OUT_OF_MEMORY, "partition slot: %s", hipGetErrorString(e)));
        x.d_col = (int32_t*)(x.mem + o_col);
        x.d_degw = (uint32_t*)(x.mem + o_degw);
        x.d_gtab_deg = (uint64_t*)(x.mem + o_gdeg);
        if (pg->has_ew) {
            x.d_ew = (uint32_t*)(x.mem + o_ew);
            x.d_gtab_ew = (uint64_t*)(x.mem + o_gew);
        }
        if ((e = hipEventCreateWithFlags(&x.ready, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&x.idle, hipEventDisableTiming)) != hipSuccess)
            return cleanup(fail(CSAW_ERR_DEVICE, "event: %s", hipGetErrorString(e)));
    }
    if ((e = hipMemcpyAsync(pg->d_vb, pg->vb.data(), (np + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        return cleanup(fail(CSAW_ERR_DEVICE, "upload: %s", hipGetErrorString(e)));
    // per-partition preparation through slot 0: the degree bias of every edge,
    // the positive counts and totals of the partition's lists, their chunk
    // prefix rows; the edge-sized results go back to pinned host memory
    auto& x = pg->slots[0];
    for (int32_t q = 0; q < np; ++q) {
        const int64_t v0 = pg->vb[q], nvq = pg->vb[q + 1] - v0, e0 = pg->eb[q], ne = pg->eb[q + 1] - e0;
        const int64_t r0 = e0 >> kTabShift, nr = pg->rows(q);
        if (ne > 0 && (e = hipMemcpyAsync(x.d_col, pg->h_col + e0, (size_t)ne * 4, hipMemcpyHostToDevice, s)) !=
                          hipSuccess)
            return cleanup(fail(CSAW_ERR_DEVICE, "upload: %s", hipGetErrorString(e)));
        launch_degree_weights(g->rowptr, x.d_col, ne, x.d_degw, s);
        if (nvq > 0) {
            launch_positive_counts(g->rowptr.shifted(v0), x.d_degw - e0, nvq, g->ppos_deg + v0, g->wtot_deg + v0, s);
            launch_chunk_table(g->rowptr.shifted(v0), x.d_degw - e0, nvq, x.d_gtab_deg - r0 * kChunkGroups, nullptr, s);
        }
        if (pg->has_ew) {
            if (ne > 0 && (e = hipMemcpyAsync(x.d_ew, pg->h_ew + e0, (size_t)ne * 4, hipMemcpyHostToDevice, s)) !=
                              hipSuccess)
                return cleanup(fail(CSAW_ERR_DEVICE, "upload: %s", hipGetErrorString(e)));
            if (nvq > 0) {
                launch_positive_counts(g->rowptr.shifted(v0), x.d_ew - e0, nvq, g->ppos_ew + v0, g->wtot_ew + v0, s);
                launch_chunk_table(g->rowptr.shifted(v0), x.d_ew - e0, nvq, x.d_gtab_ew - r0 * kChunkGroups, nullptr, s);
            }
        }
        if ((e = hipGetLastError()) != hipSuccess ||
            (ne > 0 && (e = hipMemcpyAsync(pg->h_degw + e0, x.d_degw, (size_t)ne * 4, hipMemcpyDeviceToHost, s)) !=
                           hipSuccess) ||
            (nr > 0 && (e = hipMemcpyAsync(pg->h_gtab_deg + r0 * kChunkGroups, x.d_gtab_deg,
                                           (size_t)nr * kChunkGroups * 8, hipMemcpyDeviceToHost, s)) != hipSuccess) ||
            (pg->has_ew && nr > 0 &&
             (e = hipMemcpyAsync(pg->h_gtab_ew + r0 * kChunkGroups, x.d_gtab_ew, (size_t)nr * kChunkGroups * 8,
                                 hipMemcpyDeviceToHost, s)) != hipSuccess) ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return cleanup(fail(CSAW_ERR_DEVICE, "partition preparation: %s", hipGetErrorString(e)));
    }
    // the last partition stays in slot 0 with every array
    x.part = np - 1;
    x.col = x.degw = true;
    x.ew = pg->has_ew;
    HIP_OR_FAIL(hipEventRecord(x.ready, s));
    HIP_OR_FAIL(hipEventRecord(x.idle, s));
    for (size_t k = 1; k < pg->slots.size(); ++k) {
        HIP_OR_FAIL(hipEventRecord(pg->slots[k].ready, s));
        HIP_OR_FAIL(hipEventRecord(pg->slots[k].idle, s));
    }
    *out = pg;
    return CSAW_OK;
}

csaw_status csaw_sample_streamed(csaw_pgraph pg, const csaw_sample_args* a, csaw_sample_out* out, csaw_stream stream,
                                 csaw_stream_stats* stats) {
    t_err.clear();
    if (!pg) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    std::lock_guard<std::mutex> lk(pg->mu);
    HIP_OR_FAIL(hipSetDevice(pg->g->device));
    if (stats) *stats = csaw_stream_stats{};
    Streamer st{pg, stats};
    return sample_call(pg->g, a, out, stream, nullptr, 0, &st);
}

csaw_status csaw_set_tuning(csaw_graph g, const csaw_tuning* t) {
    t_err.clear();
    if (!g || !t) return fail(CSAW_ERR_INVALID_ARG, "graph or tuning is NULL");
    if (t->bound16 < 0 || t->bound16 > 16 || t->bound32 < 0 || t->bound32 > 32)
        return fail(CSAW_ERR_INVALID_ARG, "bound16 must be in [0, 16] and bound32 in [0, 32]");
    g->bound16.store(t->bound16);
    g->bound32.store(t->bound32);
    return CSAW_OK;
}

csaw_status csaw_set_walk_guides(csaw_graph g, int32_t enable) {
    t_err.clear();
    if (!g) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    if (enable != 0 && enable != 1) return fail(CSAW_ERR_INVALID_ARG, "enable must be 0 or 1");
    g->walk_guides.store(enable);
    return CSAW_OK;
}

csaw_status csaw_get_walk_guides(csaw_graph g, int32_t* enable) {
    t_err.clear();
    if (!g || !enable) return fail(CSAW_ERR_INVALID_ARG, "graph or enable is NULL");
    *enable = g->walk_guides.load();
    return CSAW_OK;
}

csaw_status csaw_get_tuning(csaw_graph g, csaw_tuning* t) {
    t_err.clear();
    if (!g || !t) return fail(CSAW_ERR_INVALID_ARG, "graph or tuning is NULL");
    t->bound16 = g->bound16.load();
    t->bound32 = g->bound32.load();
    return CSAW_OK;
}

csaw_status csaw_autotune_sample(csaw_graph g, const csaw_sample_args* a, csaw_sample_out* out, int32_t reps,
                                 csaw_stream stream, csaw_tuning* chosen) {
    t_err.clear();
    if (!g) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    if (reps < 1 || reps > 100) return fail(CSAW_ERR_INVALID_ARG, "reps must be in [1, 100]");
    static const csaw_tuning kCandidates[] = {{0, 0}, {8, 0}, {16, 0}, {0, 32}, {8, 32}, {16, 32}};
    csaw_tuning prev;
    csaw_get_tuning(g, &prev);
    csaw_tuning best = prev;
    double best_t = 0;
    for (const csaw_tuning& c : kCandidates) {
        csaw_set_tuning(g, &c);
        std::vector<double> ts;
        for (int r = 0; r <= reps; ++r) {  // call 0 warms up (and captures this setting's graph)
            const auto t0 = std::chrono::steady_clock::now();
            const csaw_status st = csaw_sample(g, a, out, stream);  // returns after its stream drained
            const auto t1 = std::chrono::steady_clock::now();
            if (st != CSAW_OK) {
                csaw_set_tuning(g, &prev);
                return st;
            }
            if (r > 0) ts.push_back(std::chrono::duration<double>(t1 - t0).count());
        }
        std::nth_element(ts.begin(), ts.begin() + ts.size() / 2, ts.end());
        const double med = ts[ts.size() / 2];
        if (&c == kCandidates || med < best_t) {
            best_t = med;
            best = c;
        }
    }
    csaw_set_tuning(g, &best);
    if (chosen) *chosen = best;
    return CSAW_OK;
}

// One walk call; its two device counters live in a pooled workspace, or in
// `scratch` (kWalkScratchBytes of device memory) when that is set.
// Checks of a walk call's kind and thresholds, and the tables its kind
// needs: built here, or (calls in caller memory, which must not allocate)
// required to exist already.
static csaw_status walk_prepare(csaw_graph g, const csaw_walk_args* a, hipStream_t s, bool in_caller_memory) {
    if (!g) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    if (!a) return fail(CSAW_ERR_INVALID_ARG, "args is NULL");
    if (a->bias_kind < kUniform || a->bias_kind > kMetropolis) return fail(CSAW_ERR_INVALID_ARG, "bad bias kind");
    if (a->bias_kind == kEdgeWeight && !g->ew) return fail(CSAW_ERR_INVALID_ARG, "EDGE_WEIGHT bias without edge weights");
    if (a->bias_kind == kNode2vec && !g->sorted) return fail(CSAW_ERR_INVALID_ARG, "NODE2VEC needs sorted adjacency lists");
    if ((uint64_t)a->restart_threshold + (uint64_t)a->jump_threshold > (uint64_t(1) << 32))
        return fail(CSAW_ERR_INVALID_ARG, "restart_threshold + jump_threshold exceeds 2^32");
    HIP_OR_FAIL(hipSetDevice(g->device));
    if (a->bias_kind == kNode2vec) {
        // node2vec's second-order bias is defined on undirected graphs: the
        // first such walk checks on the device that every edge has its
        // reverse (no allocation: the graph's flag word), later ones reuse it
        std::lock_guard<std::mutex> lk(g->mu);
        if (g->symmetric < 0) {
            int32_t h = 0;
            HIP_OR_FAIL(hipMemsetAsync(g->dflag, 0, sizeof(int32_t), s));
            launch_symmetric_check(g->rowptr, g->col, g->n, g->dflag, s);
            HIP_OR_FAIL(hipGetLastError());
            HIP_OR_FAIL(hipMemcpyAsync(&h, g->dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIP_OR_FAIL(hipStreamSynchronize(s));
            g->symmetric = h ? 0 : 1;
        }
        if (!g->symmetric) return fail(CSAW_ERR_INVALID_ARG, "NODE2VEC needs a symmetric graph (an edge has no reverse)");
    }
    if (a->bias_kind == kNeighborDegree || a->bias_kind == kEdgeWeight) {
        if (in_caller_memory) {
            std::lock_guard<std::mutex> lk(g->mu);
            if (!(a->bias_kind == kNeighborDegree ? g->ppos_deg : g->ppos_ew))
                return fail(CSAW_ERR_NOT_READY, "the tables of this bias kind are not built yet");
        } else {
            csaw_status st = prepare_bias(g, a->bias_kind, s);
            if (st == CSAW_OK && g->walk_guides.load()) st = prepare_walk_guides(g, a->bias_kind, s);
            if (st != CSAW_OK) return st;
        }
    }
    return CSAW_OK;
}

static WalkParams walk_params(csaw_graph g, const csaw_walk_args* a) {
    WalkParams p;
    p.g = g->dev();
    p.bias = a->bias_kind;
    p.w_return = a->w_return;
    p.w_common = a->w_common;
    p.w_outward = a->w_outward;
    p.num_walkers = a->num_walkers;
    p.starts = a->starts;
    p.walker_base = a->walker_base;
    p.length = a->length;
    p.k0 = (uint32_t)a->rng_seed;
    p.k1 = (uint32_t)(a->rng_seed >> 32);
    p.walker_ids = a->walker_ids;
    p.restart = a->restart_threshold;
    p.jump = a->jump_threshold;
    p.batch = WalkBatch{};
    return p;
}

static csaw_status walk_call(csaw_graph g, const csaw_walk_args* a, int32_t* paths, int64_t* total_steps,
                             csaw_stream stream, char* scratch) {
    if (a && (a->num_walkers < 0 || a->length < 0))
        return fail(CSAW_ERR_INVALID_ARG, "negative num_walkers or length");
    if (a && a->num_walkers > 0 && (!a->starts || !paths)) return fail(CSAW_ERR_INVALID_ARG, "starts/paths is NULL");
    hipStream_t s = (hipStream_t)stream;
    csaw_status st;
    if ((st = walk_prepare(g, a, s, scratch != nullptr)) != CSAW_OK) return st;
    if (total_steps) *total_steps = 0;
    if (a->num_walkers == 0) return CSAW_OK;
    Lease rel{g, nullptr, s};
    char* dev = scratch;
    char* host = nullptr;
    uint64_t readback[kWalkScratchBytes / 8];
    if (!scratch) {
        Workspace* ws = acquire(g);
        rel.w = ws;
        if ((st = ensure_arena(ws, kWalkScratchBytes)) != CSAW_OK) return st;
        if ((st = ensure_pinned(ws, kWalkScratchBytes)) != CSAW_OK) return st;
        dev = ws->arena;
        host = ws->pinned;
    } else {
        host = (char*)readback;
    }
    unsigned long long* d_steps = (unsigned long long*)dev;
    int32_t* d_bad = (int32_t*)(dev + 256);
    HIP_OR_FAIL(hipMemsetAsync(dev, 0, kWalkScratchBytes, s));
    WalkParams p = walk_params(g, a);
    p.paths = paths;
    p.steps = d_steps;
    p.bad_start = d_bad;
    {
        ProfScope ps(a->bias_kind == kNode2vec ? "walk_node2vec" : "walk", s, true);
        launch_walk(p, 65536, s, ps.ev());
    }
    HIP_OR_FAIL(hipGetLastError());
    HIP_OR_FAIL(hipMemcpyAsync(host, dev, kWalkScratchBytes, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    rel.clean = true;
    const unsigned long long steps = *(unsigned long long*)host;
    const int32_t bad = *(int32_t*)(host + 256);
    if (bad) return fail(CSAW_ERR_INVALID_ARG, "a start vertex is outside [0, n)");
    // a device-written count: at most one step per walker and step index
    if (steps > (unsigned long long)a->num_walkers * (unsigned long long)a->length)
        return fail(CSAW_ERR_DEVICE, "the device reported %llu steps for %lld walkers of length %d", steps,
                    (long long)a->num_walkers, a->length);
    if (total_steps) *total_steps = (int64_t)steps;
    return CSAW_OK;
}

csaw_status csaw_walk(csaw_graph g, const csaw_walk_args* a, int32_t* paths, int64_t* total_steps,
                      csaw_stream stream) {
    t_err.clear();
    return walk_call(g, a, paths, total_steps, stream, nullptr);
}


csaw_status csaw_mdrw(csaw_graph g, const csaw_mdrw_args* a, int32_t* src, int32_t* dst, int64_t* steps,
                      int64_t* total_edges, csaw_stream stream) {
    t_err.clear();
    if (!g) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    if (!a) return fail(CSAW_ERR_INVALID_ARG, "args is NULL");
    if (a->num_instances < 0 || a->budget < 0) return fail(CSAW_ERR_INVALID_ARG, "negative num_instances or budget");
    const int32_t ni = a->num_instances;
    if (ni > 0 && !a->pool_offsets) return fail(CSAW_ERR_INVALID_ARG, "pool_offsets is NULL");
    if (ni > 0 && a->pool_offsets[0] != 0) return fail(CSAW_ERR_INVALID_ARG, "pool_offsets[0] != 0");
    for (int32_t i = 0; i < ni; ++i) {
        const int64_t P = a->pool_offsets[i + 1] - a->pool_offsets[i];
        if (P < 0) return fail(CSAW_ERR_INVALID_ARG, "pool_offsets decreases at %d", i);
        if (P > kMaxPool) return fail(CSAW_ERR_UNSUPPORTED, "pool %d has %lld vertices (most %d)", i, (long long)P, kMaxPool);
    }
    if (ni > 0 && a->pool_offsets[ni] > 0 && !a->pool) return fail(CSAW_ERR_INVALID_ARG, "pool is NULL");
    if ((int64_t)ni * a->budget > 0 && (!src || !dst)) return fail(CSAW_ERR_INVALID_ARG, "src/dst is NULL");
    if (total_edges) *total_edges = 0;
    hipStream_t s = (hipStream_t)stream;
    HIP_OR_FAIL(hipSetDevice(g->device));
    if (ni == 0) return CSAW_OK;
    Workspace* ws = acquire(g);
    Lease rel{g, ws, s};
    csaw_status st;
    if ((st = ensure_arena(ws, 512)) != CSAW_OK) return st;
    // pinned block: [0, 512) read-back of the counters, then the pool offsets
    const size_t o_off = 512;
    if ((st = ensure_pinned(ws, o_off + ((size_t)ni + 1) * sizeof(int64_t))) != CSAW_OK) return st;
    std::memcpy(ws->pinned + o_off, a->pool_offsets, ((size_t)ni + 1) * sizeof(int64_t));
    unsigned long long* d_total = (unsigned long long*)ws->arena;
    int32_t* d_bad = (int32_t*)(ws->arena + 256);
    HIP_OR_FAIL(hipMemsetAsync(ws->arena, 0, 512, s));
    MdrwParams p;
    p.g = g->dev();
    p.num_instances = ni;
    p.pool_off = (const int64_t*)(ws->pinned_dev + o_off);
    p.pool = a->pool;
    p.instance_base = a->instance_base;
    p.budget = a->budget;
    p.k0 = (uint32_t)a->rng_seed;
    p.k1 = (uint32_t)(a->rng_seed >> 32);
    p.src = src;
    p.dst = dst;
    p.steps = steps;
    p.total = d_total;
    p.bad = d_bad;
    {
        ProfScope ps("mdrw", s, true);
        launch_mdrw(p, s, ps.ev());
    }
    HIP_OR_FAIL(hipGetLastError());
    HIP_OR_FAIL(hipMemcpyAsync(ws->pinned, ws->arena, 512, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    rel.clean = true;
    const unsigned long long tot = *(unsigned long long*)ws->pinned;
    const int32_t bad = *(int32_t*)(ws->pinned + 256);
    if (total_edges) *total_edges = (int64_t)tot;
    if (bad) return fail(CSAW_ERR_INVALID_ARG, "a pool vertex is outside [0, n)");
    return CSAW_OK;
}

csaw_status csaw_layer_sample(csaw_graph g, const csaw_layer_args* a, int32_t* src, int32_t* dst, int32_t* counts,
                              csaw_stream stream) {
    t_err.clear();
    if (!g) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    if (!a) return fail(CSAW_ERR_INVALID_ARG, "args is NULL");
    const int32_t ni = a->num_instances, L = a->num_layers;
    if (ni < 0) return fail(CSAW_ERR_INVALID_ARG, "num_instances < 0");
    if (L < 0 || L > CSAW_MAX_LAYERS) return fail(CSAW_ERR_INVALID_ARG, "num_layers must be in [0, %d]", CSAW_MAX_LAYERS);
    if (L > 0 && !a->fanouts) return fail(CSAW_ERR_INVALID_ARG, "fanouts is NULL");
    int32_t K = 0;
    for (int32_t l = 0; l < L; ++l) {
        if (a->fanouts[l] < 1 || a->fanouts[l] > 64) return fail(CSAW_ERR_INVALID_ARG, "fanouts must be in [1, 64]");
        K = std::max(K, a->fanouts[l]);
    }
    if (a->bias_kind != kUniform && a->bias_kind != kEdgeWeight && a->bias_kind != kNeighborDegree)
        return fail(CSAW_ERR_INVALID_ARG, "bias kind %d is not a sampling bias", a->bias_kind);
    if (a->bias_kind == kEdgeWeight && !g->ew) return fail(CSAW_ERR_INVALID_ARG, "EDGE_WEIGHT bias without edge weights");
    if (a->rounds < CSAW_DIRECT_ONLY || a->rounds > CSAW_ROUNDS)
        return fail(CSAW_ERR_INVALID_ARG, "rounds must be CSAW_DIRECT_ONLY, 0 (default) or 1..%d", CSAW_ROUNDS);
    if (ni > 0 && !a->seed_offsets) return fail(CSAW_ERR_INVALID_ARG, "seed_offsets is NULL");
    if (ni > 0 && a->seed_offsets[0] != 0) return fail(CSAW_ERR_INVALID_ARG, "seed_offsets[0] != 0");
    int64_t max_f = 0;
    for (int32_t i = 0; i < ni; ++i) {
        const int64_t S = a->seed_offsets[i + 1] - a->seed_offsets[i];
        if (S < 0) return fail(CSAW_ERR_INVALID_ARG, "seed_offsets decreases at %d", i);
        if (S > kMaxPool)
            return fail(CSAW_ERR_UNSUPPORTED, "instance %d has %lld seeds (most %d)", i, (long long)S, kMaxPool);
        max_f = std::max(max_f, S);
    }
    if (ni > 0 && a->seed_offsets[ni] > 0 && !a->seeds) return fail(CSAW_ERR_INVALID_ARG, "seeds is NULL");
    if ((int64_t)ni * L > 0 && (!src || !dst || !counts)) return fail(CSAW_ERR_INVALID_ARG, "src/dst/counts is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_OR_FAIL(hipSetDevice(g->device));
    csaw_status st;
    if (a->bias_kind != kUniform && (st = prepare_bias(g, a->bias_kind, s)) != CSAW_OK) return st;
    if ((int64_t)ni * L == 0) return CSAW_OK;
    Workspace* ws = acquire(g);
    Lease rel{g, ws, s};
    if ((st = ensure_arena(ws, 512)) != CSAW_OK) return st;
    // pinned block: [0, 512) read-back of the error flag, then the seed offsets
    const size_t o_off = 512;
    if ((st = ensure_pinned(ws, o_off + ((size_t)ni + 1) * sizeof(int64_t))) != CSAW_OK) return st;
    std::memcpy(ws->pinned + o_off, a->seed_offsets, ((size_t)ni + 1) * sizeof(int64_t));
    HIP_OR_FAIL(hipMemsetAsync(ws->arena, 0, 512, s));
    LayerParams p{};
    p.g = g->dev();
    p.num_instances = ni;
    p.seed_off = (const int64_t*)(ws->pinned_dev + o_off);
    p.seeds = a->seeds;
    p.instance_base = a->instance_base;
    p.L = L;
    p.K = K;
    p.max_f = (int32_t)max_f;
    for (int32_t l = 0; l < L; ++l) p.fan[l] = a->fanouts[l];
    p.bias = a->bias_kind;
    p.rounds = a->rounds == 0 ? kDefaultRounds : (a->rounds == CSAW_DIRECT_ONLY ? 0 : a->rounds);
    p.k0 = (uint32_t)a->rng_seed;
    p.k1 = (uint32_t)(a->rng_seed >> 32);
    p.src = src;
    p.dst = dst;
    p.counts = counts;
    p.bad = (int32_t*)ws->arena;
    {
        ProfScope ps("layer_sample", s, true);
        launch_layer_sample(p, s, ps.ev());
    }
    HIP_OR_FAIL(hipGetLastError());
    HIP_OR_FAIL(hipMemcpyAsync(ws->pinned, ws->arena, 512, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    rel.clean = true;
    if (*(int32_t*)ws->pinned) return fail(CSAW_ERR_INVALID_ARG, "seeds out of range, unsorted or repeated");
    return CSAW_OK;
}

}  // extern "C"

namespace csaw {

csaw_status sample_plan_caps(csaw_graph g, const csaw_sample_args* a, std::vector<int64_t>& fcap,
                             int64_t* max_edges) {
    SamplePlan P;
    const csaw_status st = plan_sample(g, a, P, false);
    if (st != CSAW_OK) return st;
    fcap = P.fcap;
    *max_edges = P.max_edges;
    return CSAW_OK;
}

size_t sample_scratch_bytes(csaw_graph g, int32_t ni, int32_t L, const std::vector<int64_t>& fcap) {
    SampleLayout lay;
    if (!layout_sample(ni, L, fcap, bitmap_words_per_instance(g->n), lay)) return SIZE_MAX;
    return lay.scratch;
}

csaw_status sample_in_scratch(csaw_graph g, const csaw_sample_args* a, csaw_sample_out* out, hipStream_t stream,
                              char* scratch, size_t scratch_bytes) {
    t_err.clear();
    if (!scratch) return fail(CSAW_ERR_INVALID_ARG, "scratch is NULL");
    return sample_call(g, a, out, stream, scratch, scratch_bytes);
}

csaw_status walk_in_scratch(csaw_graph g, const csaw_walk_args* a, int32_t* paths, int64_t* total_steps,
                            hipStream_t stream, char* scratch) {
    t_err.clear();
    if (!scratch) return fail(CSAW_ERR_INVALID_ARG, "scratch is NULL");
    return walk_call(g, a, paths, total_steps, stream, scratch);
}

WalkBatchLayout walk_batch_layout(int32_t nreq, int64_t nw) {
    WalkBatchLayout y;
    Carver c;
    y.o_req = c.take<int32_t>((size_t)std::max<int64_t>(nw, 1));
    y.o_key = c.take<uint64_t>((size_t)std::max(nreq, 1));
    y.o_len = c.take<int32_t>((size_t)std::max(nreq, 1));
    y.o_first = c.take<int64_t>((size_t)std::max(nreq, 1));
    y.o_base = c.take<uint64_t>((size_t)std::max(nreq, 1));
    y.o_path = c.take<int64_t>((size_t)std::max(nreq, 1));
    y.o_steps = c.take<uint64_t>((size_t)std::max(nreq, 1) + 1);  // counters, then the start-vertex flag
    y.o_bad = y.o_steps + (size_t)std::max(nreq, 1) * sizeof(uint64_t);
    y.bytes = c.off;
    return y;
}

void walk_batch_image(const WalkBatchReq* reqs, int32_t nreq, const int64_t* path_offset, char* image) {
    int64_t nw = 0;
    for (int32_t q = 0; q < nreq; ++q) nw += reqs[q].num_walkers;
    const WalkBatchLayout y = walk_batch_layout(nreq, nw);
    std::memset(image, 0, y.bytes);
    int32_t* req = (int32_t*)(image + y.o_req);
    int64_t first = 0;
    for (int32_t q = 0; q < nreq; ++q) {
        ((uint64_t*)(image + y.o_key))[q] = reqs[q].rng_seed;
        ((int32_t*)(image + y.o_len))[q] = reqs[q].length;
        ((int64_t*)(image + y.o_first))[q] = first;
        ((uint64_t*)(image + y.o_base))[q] = reqs[q].walker_base;
        ((int64_t*)(image + y.o_path))[q] = path_offset[q];
        std::fill(req + first, req + first + reqs[q].num_walkers, q);
        first += reqs[q].num_walkers;
    }
}

csaw_status walk_batch_in_scratch(csaw_graph g, const csaw_walk_args* common, const WalkBatchReq* reqs,
                                  int32_t nreq, const int32_t* d_starts, int32_t* d_paths, char* d_tables,
                                  int64_t* steps, hipStream_t s) {
    t_err.clear();
    if (nreq <= 0 || !reqs || !d_tables || !steps) return fail(CSAW_ERR_INVALID_ARG, "empty walk batch");
    int64_t nw = 0;
    for (int32_t q = 0; q < nreq; ++q) {
        if (reqs[q].num_walkers < 0 || reqs[q].length < 0)
            return fail(CSAW_ERR_INVALID_ARG, "negative num_walkers or length");
        nw += reqs[q].num_walkers;
    }
    if (nw > 0 && (!d_starts || !d_paths)) return fail(CSAW_ERR_INVALID_ARG, "starts/paths is NULL");
    csaw_status st;
    if ((st = walk_prepare(g, common, s, true)) != CSAW_OK) return st;
    for (int32_t q = 0; q < nreq; ++q) steps[q] = 0;
    if (nw == 0) return CSAW_OK;
    const WalkBatchLayout y = walk_batch_layout(nreq, nw);
    WalkParams p = walk_params(g, common);
    p.num_walkers = nw;
    p.starts = d_starts;
    p.walker_ids = nullptr;
    p.paths = d_paths;
    p.steps = (unsigned long long*)(d_tables + y.o_steps);
    p.bad_start = (int32_t*)(d_tables + y.o_bad);
    p.batch.req = (const int32_t*)(d_tables + y.o_req);
    p.batch.key = (const uint64_t*)(d_tables + y.o_key);
    p.batch.length = (const int32_t*)(d_tables + y.o_len);
    p.batch.first = (const int64_t*)(d_tables + y.o_first);
    p.batch.base = (const uint64_t*)(d_tables + y.o_base);
    p.batch.path = (const int64_t*)(d_tables + y.o_path);
    p.batch.steps = (unsigned long long*)(d_tables + y.o_steps);
    {
        ProfScope ps(common->bias_kind == kNode2vec ? "walk_node2vec" : "walk", s, true);
        launch_walk(p, 65536, s, ps.ev());
    }
    HIP_OR_FAIL(hipGetLastError());
    std::vector<uint64_t> back((size_t)nreq + 1, 0);
    HIP_OR_FAIL(hipMemcpyAsync(back.data(), d_tables + y.o_steps, back.size() * sizeof(uint64_t),
                               hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    if ((int32_t)back[nreq]) return fail(CSAW_ERR_INVALID_ARG, "a start vertex is outside [0, n)");
    for (int32_t q = 0; q < nreq; ++q) {
        // a device-written count: at most one step per walker and step index
        if (back[q] > (uint64_t)reqs[q].num_walkers * (uint64_t)reqs[q].length)
            return fail(CSAW_ERR_DEVICE, "the device reported %llu steps for %lld walkers of length %d",
                        (unsigned long long)back[q], (long long)reqs[q].num_walkers, reqs[q].length);
        steps[q] = (int64_t)back[q];
    }
    return CSAW_OK;
}

csaw_status prepare_bias_tables(csaw_graph g, int32_t kind, hipStream_t stream) {
    t_err.clear();
    if (!g) return fail(CSAW_ERR_INVALID_ARG, "graph is NULL");
    if (kind == kEdgeWeight && !g->ew) return fail(CSAW_ERR_INVALID_ARG, "EDGE_WEIGHT bias without edge weights");
    if (kind != kEdgeWeight && kind != kNeighborDegree) return CSAW_OK;
    HIP_OR_FAIL(hipSetDevice(g->device));
    const csaw_status st = prepare_bias(g, kind, stream);
    return st != CSAW_OK || !g->walk_guides.load() ? st : prepare_walk_guides(g, kind, stream);
}

}  // namespace csaw

extern "C" {

csaw_status csaw_set_allocator(csaw_alloc_fn alloc_fn, csaw_free_fn free_fn, void* user) {
    t_err.clear();
    if ((alloc_fn == nullptr) != (free_fn == nullptr))
        return fail(CSAW_ERR_INVALID_ARG, "alloc_fn and free_fn must both be set or both be NULL");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc_fn;
    g_alloc.release = free_fn;
    g_alloc.user = user;
    return CSAW_OK;
}

csaw_status csaw_profile_enable(int32_t on) {
    g_prof.store(on != 0);
    return CSAW_OK;
}

csaw_status csaw_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof_recs) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_recs.clear();
    return CSAW_OK;
}

csaw_status csaw_profile_read(const char* prefix, double* total_ms, int64_t* launches) {
    if (!prefix || !total_ms || !launches) return fail(CSAW_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double t = 0;
    int64_t c = 0;
    const size_t pl = std::strlen(prefix);
    for (auto& r : g_prof_recs) {
        if (r.name.compare(0, pl, prefix) != 0) continue;
        HIP_OR_FAIL(hipEventSynchronize(r.b));
        float ms = 0;
        HIP_OR_FAIL(hipEventElapsedTime(&ms, r.a, r.b));
        t += ms;
        ++c;
    }
    *total_ms = t;
    *launches = c;
    return CSAW_OK;
}

}  // extern "C"
