// kernels.h -- host-side launchers of the gfx950 kernels (internal to libcsaw).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csaw {

constexpr int kMaxLayers = 16;
constexpr int kMaxDrawFanout = 64;   // slots of one wave
constexpr int kDefaultRounds = 8;    // repeated-sampling rounds before the direct draws
constexpr uint32_t kBurnRound = 0xFFFEu;  // counter word 3 (high half) of the forest fire trials
constexpr int32_t kBurnCapAll = 64;       // burning cap of a fanout of -1
constexpr int kChunk = 1024;         // weights per chunk of a long list
constexpr int kChunkGroups = 64;     // 16-weight groups per chunk
constexpr int32_t kWideList = (int32_t)0x80000000u;  // ppos flag: the list's total weight is >= 2^32

enum BiasKind : int32_t { kUniform = 0, kEdgeWeight = 1, kNeighborDegree = 2, kNode2vec = 3, kMetropolis = 4 };

// Graph resident in HBM.
// CSR row offsets: 32-bit words when every offset fits (m < 2^32), else
// 64-bit; v's list is [rowptr[v], rowptr[v + 1]). Exactly one pointer is set.
struct RowPtr {
    const uint32_t* p32;
    const int64_t* p64;
    __host__ __device__ __forceinline__ int64_t operator[](int64_t v) const {
        return p32 ? (int64_t)p32[v] : p64[v];
    }
    // the same offsets seen from vertex v0 on (index v means vertex v0 + v)
    RowPtr shifted(int64_t v0) const { return RowPtr{p32 ? p32 + v0 : nullptr, p64 ? p64 + v0 : nullptr}; }
    const void* data() const { return p32 ? (const void*)p32 : (const void*)p64; }
};

// One edge of the walk guide: the inclusive prefix S_(i+1) of edge i in its
// list beside the edge's neighbor and weight, so that a probe of a few
// positions reads one run of 16-byte records (a sampling draw also needs the
// exclusive prefix S_i = S_(i+1) - w and the weight of its pick).
struct alignas(16) WalkEdge {
    uint64_t S;
    int32_t col;
    uint32_t w;
};

// One vertex of the walk guide (graphs with m < 2^32): its list
// [beg, beg + d) and the list's total W in one 16-byte record.
struct alignas(16) WalkVertex {
    uint64_t W;
    uint32_t beg;
    uint32_t d;
};

// One bucket of a list's walk guide: the position i whose interval
// [S_i, S_(i+1)) holds the bucket's start, with that position's exact
// prefix S_(i+1) and neighbor, so that a bracket of one or two positions
// needs no edge record.
struct alignas(16) WalkBucket {
    uint64_t S;
    uint32_t pos;
    int32_t col;
};

struct GraphDev {
    int64_t n, m;
    RowPtr rowptr;             // n+1
    const int32_t* col;        // m
    const uint32_t* ew;        // m or null (EDGE_WEIGHT)
    const uint32_t* degw;      // m or null (NEIGHBOR_DEGREE, materialised)
    const int32_t* ppos_ew;    // n: #positive weights per list | kWideList, or null
    const int32_t* ppos_deg;   // n
    // chunk prefix tables of the lists longer than kWaveMaxD, one per weight
    // array: chunk j of the list starting at edge b is row (b >> 9) + j of
    // kChunkGroups inclusive group prefixes (built once per graph)
    const uint64_t* gtab_ew;
    const uint64_t* gtab_deg;
    const uint64_t* wtot_ew;   // n: total weight of each list, per weight array
    const uint64_t* wtot_deg;
    // running chunk totals of the same lists, one per chunk row: row
    // (b >> 9) + j holds the total of chunks 0..j (null on partitioned graphs)
    const uint64_t* ctab_ew;
    const uint64_t* ctab_deg;
    // walk guide tables (null until the first weighted walk of the weight
    // array): wrec[e] = edge e's inclusive prefix in its list and its
    // neighbor (lists with a positive total); wvtx[v] = v's list and total
    // (every vertex; null when m >= 2^32); the list v starting at edge b
    // owns the buckets wgd[2 b + v + k], k < K (at most 2 d of its 2 d + 1
    // slots; K and s from guide_shift): the first position i with
    // S_(i+1) > k * 2^s, its S_(i+1) and its neighbor
    const WalkEdge* wrec_ew;
    const WalkEdge* wrec_deg;
    const WalkVertex* wvtx_ew;
    const WalkVertex* wvtx_deg;
    const WalkBucket* wgd_ew;
    const WalkBucket* wgd_deg;
};

constexpr int kWaveMaxD = 512;   // longest weighted list of the wavefront kernels
constexpr int kTabShift = 9;     // row of a list's first chunk: first edge >> kTabShift

// Device-resident control block of one sampling call.
struct SampleCtl {
    int64_t fcount[kMaxLayers + 1];    // frontier sizes
    int64_t total[kMaxLayers];         // edges per layer
    int64_t out_base[kMaxLayers + 1];  // first edge of each layer
    unsigned long long nbig[kMaxLayers];    // long weighted lists per layer
    int64_t ndirty[kMaxLayers + 1];    // dirty words per layer (sparse builds)
    int32_t bad_seed;
    int32_t overflow;
    int32_t unsupported;
    int32_t lookback_stuck;
};

static_assert(sizeof(SampleCtl) % 4 == 0, "control block is copied in 32-bit words");

// One frontier build: next bitmap -> sorted frontier entries with their edge
// counts, edge offsets, kernel routes and per-instance segment offsets.
struct FrontierBuild {
    GraphDev g;
    uint32_t* next;
    uint32_t* visited;
    int64_t nwords;                  // words of all instances' bitmaps
    int64_t nwp;                     // words per instance
    int64_t nb;                      // blocks of the launch
    int32_t layer;
    int32_t num_layers;
    int32_t num_instances;
    const int32_t* fanout;           // [ni] fanout of this layer
    const int32_t* bias;             // [ni]
    const uint32_t* inst_id;         // [ni] instance id mod 2^32 (forest fire counters)
    const uint64_t* inst_key;        // [ni] Philox key per instance
    uint32_t burn;                   // forest fire threshold (0: fixed fanout)
    int32_t* fv;
    int32_t* fi;
    int32_t* cnt;
    int64_t* off;
    int64_t* fbeg;                   // per entry: first edge of its list
    int32_t* fdeg;                   // per entry: list length
    int32_t* fpos;                   // per entry: positive biases | kWideList (list length if unbiased)
    int32_t* bigs;                   // long-list entries (frontier positions)
    int64_t* offsets;                // [L*ni+1] or null
    SampleCtl* ctl;
    unsigned long long* status;      // [4 * max(nb, nb_dirty)] look-back words
    // sparse build (large bitmaps): summary bitmap, one bit per next word
    // (nsw words per instance, a multiple of 4), and the dirty-word list
    uint32_t* summ;                  // null: dense build over every word
    int64_t nsw;
    int64_t* dirty;                  // [frontier capacity]
    int64_t nb_dirty;                // blocks of the compaction
};

struct SampleLayer {
    GraphDev g;
    int32_t layer;
    int32_t num_instances;
    const uint32_t* inst_id;         // [ni] instance id mod 2^32 (counter word 0)
    const uint64_t* inst_key;        // [ni] Philox key per instance
    const int32_t* fanout;           // [ni] fanout of this layer per instance
    const int32_t* fanout_next;      // [ni] fanout of the next layer (0 = none)
    const int32_t* bias;             // [ni]
    const int32_t* fv;               // frontier vertices
    const int32_t* fi;               // frontier instance indices
    const int32_t* cnt;              // per-entry edge count
    const int64_t* off;              // per-entry exclusive offset
    const int64_t* fbeg;             // per-entry first edge of its list
    const int32_t* fdeg;             // per-entry list length
    const int32_t* fpos;             // per-entry positive biases | kWideList
    const int32_t* bigs;             // long weighted lists (frontier positions)
    SampleCtl* ctl;
    int32_t* src;
    int32_t* dst;
    int64_t capacity;
    const uint32_t* visited;         // [ni * nwp]
    uint32_t* next;                  // [ni * nwp]
    int64_t nwp;                     // bitmap words per instance (multiple of 4)
    uint32_t* summ;                  // [ni * nsw] summary bitmap of next (sparse builds) or null
    int64_t nsw;
    int32_t group16, group32;        // sub-wave bucket bounds (<= 16, <= 32; 0 = off)
    int32_t rounds;                  // repeated-sampling rounds (0: every slot by direct draw)
    uint32_t burn;                   // forest fire threshold (0: fixed fanout)
    int32_t vlo, vhi;                // entries of vertices in [vlo, vhi) only (out-of-memory schedule)
};

constexpr int32_t kDefaultBound16 = 16, kDefaultBound32 = 32;

// Optional events that a launch fills with its kernel's own start and stop
// times (hipExtLaunchKernel), for kernel timing without dispatch latency.
// Only profiled calls pass them; those run eagerly, never under capture.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

template <class... A>
inline void launch_kernel(void (*kernel)(A...), dim3 grid, dim3 block, hipStream_t s, LaunchEvents ev, A... args) {
    if (ev.start || ev.stop) hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev.start, ev.stop, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// --- sampling (sample_kernels.hip)
void launch_mark_seeds(const int32_t* seeds, int64_t num_seeds, const int64_t* seed_offsets,
                       int32_t ni, int64_t n, uint32_t* next, int64_t nwp, uint32_t* summ, int64_t nsw,
                       SampleCtl* ctl, hipStream_t s);
int64_t frontier_build_blocks(int64_t words);
int64_t dirty_compact_blocks(int64_t summary_words);
int64_t sparse_build_blocks(int64_t capacity);
// Bitmap words (all instances) above which frontier builds are sparse.
constexpr int64_t kSparseWords = int64_t(1) << 23;
void launch_frontier_build(const FrontierBuild& fb, hipStream_t s, LaunchEvents ev = {});
void launch_select(const SampleLayer& p, int grid, hipStream_t s, LaunchEvents ev = {});
void launch_select_small(const SampleLayer& p, int grid, hipStream_t s, LaunchEvents ev = {});
// Chunk prefix table of every list longer than kWaveMaxD (GraphDev::gtab_*),
// rows ((m >> kTabShift) + 1) * kChunkGroups uint64.
int64_t chunk_table_rows(int64_t m);
void launch_chunk_table(RowPtr rowptr, const uint32_t* w, int64_t n, uint64_t* tab, uint64_t* ctab,
                        hipStream_t s);
void launch_select_big(const SampleLayer& p, int grid, hipStream_t s, LaunchEvents ev = {});
// Clears the visited bits of every frontier entry of the call's layers.
struct ClearVisited {
    const int32_t* fv[kMaxLayers + 1];
    const int32_t* fi[kMaxLayers + 1];
    const int64_t* fcount;           // device: entries per layer
    const SampleCtl* ctl;            // final control block of the call ...
    SampleCtl* host_ctl;             // ... copied here (host memory, device address)
    int32_t num_layers;
    int64_t cap_entries;             // largest frontier capacity (grid sizing)
    uint32_t* visited;
    int64_t nwp;
};
void launch_clear_visited(const ClearVisited& c, hipStream_t s, LaunchEvents ev = {});
// Start of a call: zero ctl[0, nctl) and copy tab[0, ntab) words from host memory.
void launch_call_setup(uint32_t* ctl, int64_t nctl, const uint32_t* host_tab, uint32_t* tab, int64_t ntab,
                       hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);
// Segment j = edges [off[j], off[j+1]) of src / dst to to_src[j] / to_dst[j]
// (device addresses, null: skipped); off is device memory, non-decreasing,
// with off[0] = 0 and off[nseg] = total.
void launch_scatter_segments(const int32_t* src, const int32_t* dst, const int64_t* off, int64_t nseg,
                             int64_t total, int32_t* const* to_src, int32_t* const* to_dst, hipStream_t s);
// Out-of-memory schedule: work[2p] = frontier entries and work[2p+1] = their
// edges in partition p (vertices [bounds[p], bounds[p+1])), accumulated.
constexpr int kMaxPartitionsHost = 64;
void launch_partition_work(const int32_t* fv, const int32_t* cnt, const SampleCtl* ctl, int32_t layer,
                           int64_t capacity, const int64_t* bounds, int32_t np, unsigned long long* work,
                           hipStream_t s);

// --- graph preparation (sample_kernels.hip)
void launch_degree_weights(RowPtr rowptr, const int32_t* col, int64_t m, uint32_t* degw,
                           hipStream_t s);
void launch_positive_counts(RowPtr rowptr, const uint32_t* w, int64_t n, int32_t* ppos, uint64_t* wtot,
                            hipStream_t s);

// --- walks (walk_kernels.hip)
// Several walk requests of one bias kind in one launch: walker w belongs to
// request req[w], whose Philox key, length, first walker, walker id of that
// first walker and first path entry are given per request; steps are counted
// per request. req == null: the launch is the one request of WalkParams.
struct WalkBatch {
    const int32_t* req;              // [nw] request of each walker
    const uint64_t* key;             // [nreq] Philox key (rng seed)
    const int32_t* length;           // [nreq]
    const int64_t* first;            // [nreq] first walker of the request
    const uint64_t* base;            // [nreq] walker id of that walker
    const int64_t* path;             // [nreq] first path entry (int32 units)
    unsigned long long* steps;       // [nreq] device counters
};

struct WalkParams {
    GraphDev g;
    int32_t bias;
    uint32_t w_return, w_common, w_outward;
    int64_t num_walkers;
    const int32_t* starts;
    uint64_t walker_base;
    int32_t length;
    uint32_t k0, k1;
    const uint64_t* walker_ids;      // [nw] or null
    uint32_t restart, jump;          // per-step move thresholds over [0, 2^32)
    int32_t* paths;
    unsigned long long* steps;       // device counter
    int32_t* bad_start;              // device flag
    WalkBatch batch;                 // batch.req null: a single request
};
void launch_walk(const WalkParams& p, int grid, hipStream_t s, LaunchEvents ev = {});
// The walk guide tables of weight array w (list totals wtot): rec[m],
// vtx[n] (may be null), gd[2 m + n].
void launch_walk_guides(RowPtr rowptr, const int32_t* col, const uint32_t* w, const uint64_t* wtot, int64_t n,
                        WalkEdge* rec, WalkVertex* vtx, WalkBucket* gd, hipStream_t s);
constexpr int kGuideBucketsPerEdge = 2;  // a list of d edges gets at most 2 d buckets

// Buckets of a list's walk guide: width 2^s, K = ((W - 1) >> s) + 1 of them,
// s the smallest shift that keeps K within kGuideBucketsPerEdge * d (d >= 1,
// W > 0). A draw r lies in bucket r >> s, whose entry and the next one's
// bracket the positions that can hold it; with buckets no wider than the
// list's mean weight a bracket holds about two positions on average
// whatever the weights are. Shared by the table builder and the walk steps.
__host__ __device__ __forceinline__ int guide_shift(uint64_t W, int64_t d) {
    const uint64_t kmax = (uint64_t)d * kGuideBucketsPerEdge, top = W - 1;
    if (top < kmax) return 0;
    // bit lengths: top >> s < kmax needs s >= len(top) - len(kmax), and at
    // most one more
    int s = (64 - __builtin_clzll(top)) - (64 - __builtin_clzll(kmax));
    if (s < 0) s = 0;
    while ((top >> s) >= kmax) ++s;
    return s;
}
// Entry 0 of list v's guide (first edge b).
__host__ __device__ __forceinline__ int64_t guide_base(int64_t b, int64_t v) { return kGuideBucketsPerEdge * b + v; }
// Sets *flag to 1 if some edge (u, x) has no reverse edge (x, u); lists must
// be sorted (each reverse edge is found by binary search).
void launch_symmetric_check(RowPtr rowptr, const int32_t* col, int64_t n, int32_t* flag, hipStream_t s);

// --- multi-dimensional random walk (mdrw_kernels.hip)
constexpr int kMaxPool = 2048;

// Layer sampling: one wavefront per instance; its frontier (at most
// kMaxPool seeds, then at most 64 picks per layer) and visited list in LDS,
// sized by the call's largest seed set.
struct LayerParams {
    GraphDev g;
    int32_t num_instances;
    const int64_t* seed_off;         // [ni+1] (host memory, device address)
    const int32_t* seeds;            // sorted and distinct per instance (checked)
    uint64_t instance_base;
    int32_t L, K;                    // layers, largest fanout (output row length)
    int32_t max_f;                   // largest seed set of the call (sizes the LDS)
    int32_t fan[kMaxLayers];         // 1..64
    int32_t bias;                    // kUniform, kEdgeWeight or kNeighborDegree
    int32_t rounds;
    uint32_t k0, k1;
    int32_t* src;                    // [ni, L, K]
    int32_t* dst;
    int32_t* counts;                 // [ni, L]
    int32_t* bad;
};
void launch_layer_sample(const LayerParams& p, hipStream_t s, LaunchEvents ev = {});
struct MdrwParams {
    GraphDev g;
    int32_t num_instances;
    const int64_t* pool_off;         // [ni+1], host-mapped memory
    const int32_t* pool;
    uint64_t instance_base;
    int64_t budget;
    uint32_t k0, k1;
    int32_t* src;
    int32_t* dst;
    int64_t* steps;                  // [ni] or null
    unsigned long long* total;       // device counter
    int32_t* bad;                    // device flag
};
void launch_mdrw(const MdrwParams& p, hipStream_t s, LaunchEvents ev = {});

}  // namespace csaw
