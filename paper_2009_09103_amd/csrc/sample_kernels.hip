// sample_kernels.hip -- gfx950 kernels of neighbor sampling.
//
// One layer of the generic sampling loop (fig:api(b), lines 5-8) is
//   count    : per frontier entry, how many edges it will emit (min(k, P))
//   scan     : exclusive offsets of those counts (output position per entry)
//   select   : one wavefront per frontier vertex: EdgeBias, exact uint64
//              prefix sum, Philox draws, inverse transform search, collision
//              rounds, direct draw from the updated prefix; writes the edges
//              and marks new neighbors in the instance's "next" bitmap
//   compact  : next bitmap -> sorted next frontier; visited |= next
// Frontier entries are (vertex, instance) pairs sorted by (instance, vertex),
// so edges come out in (layer, instance, source, slot) order without a sort.
#include "device_common.h"
#include "kernels.h"

namespace csaw {

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

inline int grid_for(int64_t items, int per_block, int cap = 1 << 20) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ----------------------------------------------------------- block helpers
// Exclusive scan of one int64 per thread over a block of kThreads threads;
// returns the exclusive prefix and writes the block total to *total. Every
// thread of the block must call it.
template <int kThreads = kBlock>
__device__ __forceinline__ int64_t block_excl_scan_i64(int64_t x, int64_t* total) {
    constexpr int kW = kThreads / kWave;
    __shared__ int64_t wsum[kW];
    const int lane = lane_id();
    const int wid = threadIdx.x / kWave;
    const uint64_t incl = wave_incl_scan_u64((uint64_t)x);
    if (lane == kWave - 1) wsum[wid] = (int64_t)incl;
    __syncthreads();
    int64_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kW; ++w) {
        const int64_t s = wsum[w];
        if (w < wid) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + (int64_t)incl - x;
}

__device__ __forceinline__ int popc4(uint4 w) {
    return __popc(w.x) + __popc(w.y) + __popc(w.z) + __popc(w.w);
}

// ------------------------------------------------------------------ misc
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_degree_weights(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                 int64_t m, uint32_t* __restrict__ degw) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = col[e];
        degw[e] = (uint32_t)(rowptr[x + 1] - rowptr[x]);
    }
}

// one wavefront per vertex: number of positive weights in its list
__global__ void k_positive_counts(const int64_t* __restrict__ rowptr, const uint32_t* __restrict__ w,
                                  int64_t n, int32_t* __restrict__ ppos) {
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t v = blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave; v < n; v += waves) {
        const int64_t b = rowptr[v], e = rowptr[v + 1];
        int64_t c = 0;
        for (int64_t i = b + lane; i < e; i += kWave) c += (w[i] > 0);
        c = wave_sum_i64(c);
        if (lane == 0) ppos[v] = (int32_t)c;
    }
}

// ------------------------------------------------------------- frontier
// Seeds -> next bitmap of their instance (instance of seed s: the largest i
// with seed_offsets[i] <= s).
__global__ void k_mark_seeds(const int32_t* __restrict__ seeds, int64_t num_seeds,
                             const int64_t* __restrict__ seed_off, int32_t ni, int64_t n,
                             uint32_t* __restrict__ next, int64_t nwp, SampleCtl* ctl) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < num_seeds;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = seeds[s];
        if (v < 0 || (int64_t)v >= n) {
            ctl->bad_seed = 1;
            continue;
        }
        int32_t lo = 0, hi = ni;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (seed_off[mid] <= s) lo = mid;
            else hi = mid;
        }
        atomicOr(&next[(int64_t)lo * nwp + (v >> 5)], 1u << (v & 31));
    }
}

// Bitmap compaction, pass 1: set bits per block of 256 x 4 words.
__global__ void k_bm_count(const uint4* __restrict__ next4, int64_t n4, int64_t* __restrict__ blocksum) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    int64_t c = 0;
    if (i < n4) c = popc4(next4[i]);
    int64_t tot;
    block_excl_scan_i64(c, &tot);
    if (threadIdx.x == 0) blocksum[blockIdx.x] = tot;
}

// Exclusive scan of nb block sums in place by one 1024-thread block; each
// thread owns a contiguous segment. *total receives the sum.
__global__ void __launch_bounds__(1024) k_scan_blocksums(int64_t* __restrict__ bs, int64_t nb,
                                                         const int64_t* __restrict__ nb_from_count,
                                                         int64_t items_per_block, int64_t* total) {
    if (nb_from_count) {
        const int64_t items = *nb_from_count;
        const int64_t used = (items + items_per_block - 1) / items_per_block;
        if (used < nb) nb = used;
    }
    const int t = threadIdx.x;
    const int64_t seg = (nb + 1023) / 1024;
    const int64_t b0 = t * seg, b1 = (b0 + seg < nb) ? b0 + seg : nb;
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += bs[b];
    int64_t tot;
    int64_t run = block_excl_scan_i64<1024>(s, &tot);
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t x = bs[b];
        bs[b] = run;
        run += x;
    }
    if (t == 0) *total = tot;
}

// Bitmap compaction, pass 2: emit (vertex, instance) for every set bit in
// (instance, word, bit) order; visited |= next; next = 0; record where each
// instance's entries start.
__global__ void k_bm_emit(uint4* __restrict__ next4, uint4* __restrict__ visited4, int64_t n4,
                          int64_t nwp4, const int64_t* __restrict__ blocksum, int32_t* __restrict__ fv,
                          int32_t* __restrict__ fi, int64_t* __restrict__ fstart) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    uint4 w = make_uint4(0, 0, 0, 0);
    if (i < n4) w = next4[i];
    int64_t tot;
    int64_t pos = blocksum[blockIdx.x] + block_excl_scan_i64(popc4(w), &tot);
    if (i >= n4) return;
    const int64_t inst = i / nwp4;
    const int64_t local4 = i - inst * nwp4;
    if (local4 == 0) fstart[inst] = pos;
    if ((w.x | w.y | w.z | w.w) == 0) return;
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t bits = ws[q];
        const int32_t vbase = (int32_t)((local4 * 4 + q) * 32);
        while (bits) {
            const int b = __ffs(bits) - 1;
            fv[pos] = vbase + b;
            fi[pos] = (int32_t)inst;
            ++pos;
            bits &= bits - 1;
        }
    }
    uint4 vis = visited4[i];
    vis.x |= w.x; vis.y |= w.y; vis.z |= w.z; vis.w |= w.w;
    visited4[i] = vis;
    next4[i] = make_uint4(0, 0, 0, 0);
}

// ------------------------------------------------------------------ count
// Weighted lists that need draws are routed by length: up to kWaveMaxD to the
// wavefront kernel (list resident in a per-wave LDS tile), up to kMidMaxD to
// the mid kernel (one block per list, whole list resident in LDS), longer ones
// to the hub kernel (one block per list, coarse prefix only).
constexpr int kWaveMaxD = 1024;
constexpr int kMidMaxD = 8192;

enum { kRouteWave = 0, kRouteMid = 1, kRouteHub = 2 };

__device__ __forceinline__ int route_of(int32_t kind, int32_t k, int32_t P, int64_t d) {
    if (kind == kUniform || k <= 0 || k >= P || d <= kWaveMaxD) return kRouteWave;
    return d <= kMidMaxD ? kRouteMid : kRouteHub;
}

__device__ __forceinline__ int32_t positive_count(const GraphDev& g, int32_t kind, int32_t v, int64_t d) {
    if (kind == kUniform) return (int32_t)d;
    return kind == kEdgeWeight ? g.ppos_ew[v] : g.ppos_deg[v];
}

__global__ void k_count(SampleLayer p, int32_t* __restrict__ cnt) {
    const int64_t fcount = p.ctl->fcount[p.layer];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < fcount;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = p.fv[e];
        const int32_t i = p.fi[e];
        const int32_t k = p.fanout[i];
        const int32_t kind = p.bias[i];
        const int64_t d = p.g.rowptr[v + 1] - p.g.rowptr[v];
        const int32_t P = positive_count(p.g, kind, v, d);
        int32_t c;
        if (k == 0 || P == 0) c = 0;
        else if (k < 0 || k >= P) c = P;
        else if (k > kMaxDrawFanout) {
            p.ctl->unsupported = 1;
            c = 0;
        } else {
            c = k;
            const int route = route_of(kind, k, P, d);
            if (route == kRouteMid) {
                const unsigned long long h = atomicAdd(&p.ctl->nmid[p.layer], 1ull);
                p.mids[h] = (int32_t)e;
            } else if (route == kRouteHub) {
                const unsigned long long h = atomicAdd(&p.ctl->nhub[p.layer], 1ull);
                p.hubs[h] = (int32_t)e;
            }
        }
        cnt[e] = c;
    }
}

// scan of counts: per-block sums, then apply
__global__ void k_scan_reduce(const int32_t* __restrict__ cnt, const int64_t* __restrict__ fcount_p,
                              int64_t* __restrict__ blocksum) {
    const int64_t fcount = *fcount_p;
    const int64_t b0 = blockIdx.x * (int64_t)kScanItems;
    if (b0 >= fcount) return;
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t e = b0 + threadIdx.x * 4 + q;
        if (e < fcount) s += cnt[e];
    }
    int64_t tot;
    block_excl_scan_i64(s, &tot);
    if (threadIdx.x == 0) blocksum[blockIdx.x] = tot;
}

__global__ void k_scan_apply(const int32_t* __restrict__ cnt, const int64_t* __restrict__ fcount_p,
                             const int64_t* __restrict__ blocksum, int64_t* __restrict__ off) {
    const int64_t fcount = *fcount_p;
    const int64_t b0 = blockIdx.x * (int64_t)kScanItems;
    if (b0 >= fcount) return;
    int32_t c[4];
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t e = b0 + threadIdx.x * 4 + q;
        c[q] = e < fcount ? cnt[e] : 0;
        s += c[q];
    }
    int64_t tot;
    int64_t run = blocksum[blockIdx.x] + block_excl_scan_i64(s, &tot);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t e = b0 + threadIdx.x * 4 + q;
        if (e < fcount) off[e] = run;
        run += c[q];
    }
}

// ----------------------------------------------------------------- select
// Prefix layout used by the inverse transform search of a weighted list:
// groups of g consecutive candidates (g = 16 in the wavefront path, 16 * 2^p
// in the hub path); C[t] = S[t*g] (exclusive prefix at the group starts) and
// C[nc] = W live in LDS. A search finds the group by binary search in C and
// the candidate by scanning the group's g weights (from the LDS tile when the
// whole list is resident there, otherwise from global memory / L2).
//
// Weights reach LDS in tiles of 1024: 16 coalesced loads per lane are issued
// together, stored transposed (element i at i + i/16, so that lane L's 16
// consecutive elements sit in 16 distinct banks), summed per lane, and one
// 64-lane scan turns the 64 group sums of a tile into 64 entries of C.
constexpr int kTile = 1024;
constexpr int kTilePad = kTile + kTile / 16;
constexpr int kWaveC = kWaveMaxD / 16;     // coarse entries per wavefront
constexpr int kMidThreads = 256;
constexpr int kMidWaves = kMidThreads / kWave;
constexpr int kHubThreads = 512;
constexpr int kHubWaves = kHubThreads / kWave;
constexpr int kHubC = 8192;                // coarse entries per hub block

__device__ __forceinline__ int tpad(int i) { return i + (i >> 4); }

struct CoarsePool {
    const uint64_t* C;      // LDS, nc + 1 entries
    int64_t nc;             // groups
    int64_t g;              // group length
    int64_t d;              // list length
    const uint32_t* w;      // weights of the list in global memory
    const uint32_t* tile;   // LDS tile holding the whole list, or null
};

// m = max{i in [0,d) : S_i <= r} with S_m and b_m; per lane. kResident: the
// group's weights are read from the LDS copy of the list (pl.tile), otherwise
// 16 at a time from global memory.
template <bool kResident>
__device__ __forceinline__ void coarse_search(const CoarsePool& pl, uint64_t r, int64_t& m, uint64_t& Sm,
                                              uint32_t& bm) {
    int64_t lo = 0, hi = pl.nc;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (pl.C[mid] <= r) lo = mid;
        else hi = mid;
    }
    uint64_t acc = pl.C[lo];
    int64_t i = lo * pl.g;
    const int64_t end = (i + pl.g < pl.d) ? i + pl.g : pl.d;
    m = i;
    Sm = acc;
    bm = 0;
    if (kResident) {  // g == 16: one batch of LDS reads
        uint32_t x[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) x[q] = i + q < end ? pl.tile[tpad((int)(i + q))] : 0u;
        bool found = false;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (!found && i + q < end) {
                if (acc + x[q] > r) {
                    m = i + q;
                    Sm = acc;
                    bm = x[q];
                    found = true;
                } else {
                    acc += x[q];
                }
            }
        }
        return;
    }
    for (; i < end; i += 16) {
        uint32_t x[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) x[q] = i + q < end ? pl.w[i + q] : 0u;
        bool found = false;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (!found && i + q < end) {
                if (acc + x[q] > r) {
                    m = i + q;
                    Sm = acc;
                    bm = x[q];
                    found = true;
                } else {
                    acc += x[q];
                }
            }
        }
        if (found) break;
    }
}

// Draw k distinct candidates with one lane per slot (lane j = slot j < k):
// repeated-sampling rounds where the lowest slot wins a collision, then
// direct draws from the prefix without the held candidates, in slot order.
// search(r, m, Sm, bm) is the per-lane inverse transform search.
//
// Collisions: with own != null (lists of at most kWaveMaxD candidates) an
// LDS array holds, per position, -1 once held, else the lowest open slot
// that picked it this round (ds_min); otherwise each open slot compares with
// every slot through lane reads.
template <class Search>
__device__ __forceinline__ int64_t draw_slots(Key key, uint32_t c0, uint32_t c1, uint32_t c2, int32_t k,
                                              uint64_t W, const Search& search, int32_t* own = nullptr) {
    const int lane = lane_id();
    const bool active = lane < k;
    bool held = false;
    int64_t pos = 0;
    uint64_t Spos = 0;
    uint32_t bpos = 0;
    for (int a = 0; a < kRounds; ++a) {
        const bool open = active && !held;
        if (ballot(open) == 0) break;
        int64_t m = -1;
        uint64_t Sm = 0;
        uint32_t bm = 0;
        if (open) search(draw(key, c0, c1, c2, (uint32_t)lane | ((uint32_t)a << 16), W), m, Sm, bm);
        bool reject = false;
        if (own) {
            wave_lds_sync();
            if (open) atomicMin(&own[m], lane);
            wave_lds_sync();
            reject = open && own[m] != lane;
            wave_lds_sync();
            if (open && !reject) own[m] = -1;
        } else {
            const uint64_t heldmask = ballot(held);
            const int64_t val = held ? pos : m;
            for (int q = 0; q < k; ++q) {
                const int64_t pq = readlane_i64(val, q);
                const bool qheld = (heldmask >> q) & 1ull;
                if (q != lane && pq == m && (qheld || q < lane)) reject = true;
            }
        }
        if (open && !reject) {
            held = true;
            pos = m;
            Spos = Sm;
            bpos = bm;
        }
    }
    const uint64_t heldmask = ballot(held);
    uint64_t openmask = ballot(active) & ~heldmask;
    if (openmask) {
        // before = total bias of held candidates at smaller positions
        uint64_t before = 0;
        for (uint64_t hm = heldmask; hm; hm &= hm - 1) {
            const int q = __ffsll((unsigned long long)hm) - 1;
            const int64_t pq = readlane_i64(pos, q);
            const uint32_t bq = readlane_u32(bpos, q);
            if (held && pq < pos) before += bq;
        }
        uint64_t removed = wave_sum_u64(held ? (uint64_t)bpos : 0ull);
        while (openmask) {
            const int j = __ffsll((unsigned long long)openmask) - 1;
            const uint64_t r0 = draw(key, c0, c1, c2, (uint32_t)j | (kFallbackRound << 16), W - removed);
            // skip map: every held region starting at or below the updated-prefix
            // position r0 (shifted by the held mass before it) is stepped over
            const uint64_t r = r0 + wave_sum_u64((held && Spos - before <= r0) ? (uint64_t)bpos : 0ull);
            int64_t m = 0;
            uint64_t Sm = 0;
            uint32_t bm = 0;
            search(r, m, Sm, bm);  // same r on every lane
            m = readlane_i64(m, j);
            Sm = readlane_u64(Sm, j);
            bm = readlane_u32(bm, j);
            const uint64_t bef_new = wave_sum_u64((held && pos < m) ? (uint64_t)bpos : 0ull);
            if (held && pos > m) before += bm;
            if (lane == j) {
                held = true;
                pos = m;
                Spos = Sm;
                bpos = bm;
                before = bef_new;
            }
            removed += bm;
            openmask &= openmask - 1;
        }
    }
    return pos;
}

__device__ __forceinline__ void claim(bool do_claim, const uint32_t* visb, uint32_t* nextb, int32_t x) {
    if (!do_claim) return;
    const uint32_t bit = 1u << (x & 31);
    if (!(visb[x >> 5] & bit)) atomicOr(&nextb[x >> 5], bit);
}

// Load one tile of up to 1024 weights (from list offset base) into an LDS
// tile and return this lane's sum of its 16 consecutive elements.
__device__ __forceinline__ uint64_t tile_group_sums(const uint32_t* __restrict__ w, int64_t base, int64_t d,
                                                    uint32_t* tile) {
    const int lane = lane_id();
    uint32_t x[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int64_t idx = base + c * kWave + lane;
        x[c] = idx < d ? w[idx] : 0u;
    }
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < 16; ++c) tile[tpad(c * kWave + lane)] = x[c];
    wave_lds_sync();
    uint64_t s = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) s += tile[tpad(lane * 16 + q)];
    return s;
}

struct EntryInfo {
    int32_t c, v, inst, k, kind, P;
    int64_t o, beg, d;
    bool do_claim;
};

__device__ __forceinline__ bool load_entry(const SampleLayer& p, int64_t e, int64_t out_base, EntryInfo& E) {
    E.c = uniform_i32(p.cnt[e]);
    if (E.c == 0) return false;
    E.v = uniform_i32(p.fv[e]);
    E.inst = uniform_i32(p.fi[e]);
    E.o = out_base + uniform_i64(p.off[e]);
    E.k = uniform_i32(p.fanout[E.inst]);
    E.kind = uniform_i32(p.bias[E.inst]);
    E.do_claim = p.fanout_next[E.inst] != 0;
    E.beg = uniform_i64(p.g.rowptr[E.v]);
    E.d = uniform_i64(p.g.rowptr[E.v + 1]) - E.beg;
    E.P = E.kind == kUniform ? (int32_t)E.d
                             : uniform_i32(E.kind == kEdgeWeight ? p.g.ppos_ew[E.v] : p.g.ppos_deg[E.v]);
    return true;
}

__device__ __forceinline__ void emit_slots(const SampleLayer& p, const EntryInfo& E, int64_t pos) {
    const int lane = lane_id();
    if (lane < E.k) {
        const int32_t x = p.g.col[E.beg + pos];
        p.src[E.o + lane] = E.v;
        p.dst[E.o + lane] = x;
        claim(E.do_claim, p.visited + (int64_t)E.inst * p.nwp, p.next + (int64_t)E.inst * p.nwp, x);
    }
}

__device__ void select_entry(const SampleLayer& p, int64_t e, int64_t out_base, uint32_t* tile, uint64_t* C,
                             int32_t* own) {
    const int lane = lane_id();
    EntryInfo E;
    if (!load_entry(p, e, out_base, E)) return;
    if (E.o + E.c > p.capacity) {
        if (lane == 0) p.ctl->overflow = 1;
        return;
    }
    if (route_of(E.kind, E.k, E.P, E.d) != kRouteWave) return;  // mid / hub kernels
    const uint32_t* visb = p.visited + (int64_t)E.inst * p.nwp;
    uint32_t* nextb = p.next + (int64_t)E.inst * p.nwp;
    const bool weighted = E.kind != kUniform;
    const uint32_t* w = weighted ? (E.kind == kEdgeWeight ? p.g.ew : p.g.degw) + E.beg : nullptr;
    const int32_t* col = p.g.col + E.beg;
    int32_t* src = p.src + E.o;
    int32_t* dst = p.dst + E.o;
    const int64_t d = E.d;

    // ---- NeighborSize >= pool: every positive-bias neighbor, list order
    if (E.k < 0 || E.k >= E.P) {
        if (!weighted || E.P == d) {
            for (int64_t j = lane; j < d; j += kWave) {
                const int32_t x = col[j];
                src[j] = E.v;
                dst[j] = x;
                claim(E.do_claim, visb, nextb, x);
            }
        } else {
            int64_t run = 0;
            for (int64_t base = 0; base < d; base += 8 * kWave) {
                uint32_t x[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int64_t idx = base + c * kWave + lane;
                    x[c] = idx < d ? w[idx] : 0u;
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int64_t idx = base + c * kWave + lane;
                    const bool pos = x[c] > 0;
                    const uint64_t mask = ballot(pos);
                    if (pos) {
                        const int64_t slot = run + __popcll(mask & lanemask_lt());
                        const int32_t nb = col[idx];
                        src[slot] = E.v;
                        dst[slot] = nb;
                        claim(E.do_claim, visb, nextb, nb);
                    }
                    run += __popcll(mask);
                }
            }
        }
        return;
    }

    // ---- k < P <= d: draw k distinct candidates (k <= kMaxDrawFanout)
    const Key key{p.k0, p.k1};
    const uint32_t c0 = (uint32_t)(p.instance_base + (uint64_t)E.inst);
    const uint32_t c1 = (uint32_t)p.layer;
    const uint32_t c2 = (uint32_t)E.v;
    int64_t pos;
    int32_t* ownp = nullptr;
    if (d <= kWaveMaxD) {
        for (int64_t i = lane; i < d; i += kWave) own[i] = kWave;
        ownp = own;
    }
    if (!weighted) {
        pos = draw_slots(key, c0, c1, c2, E.k, (uint64_t)d,
                         [](uint64_t r, int64_t& m, uint64_t& Sm, uint32_t& bm) {
                             m = (int64_t)r;
                             Sm = r;
                             bm = 1;
                         },
                         ownp);
    } else {
        uint64_t carry = 0;
        if (lane == 0) C[0] = 0;
        for (int64_t t = 0; t * kTile < d; ++t) {
            const uint64_t s = tile_group_sums(w, t * kTile, d, tile);
            const uint64_t incl = wave_incl_scan_u64(s);
            C[t * kWave + lane + 1] = carry + incl;
            carry += readlane_u64(incl, kWave - 1);
        }
        wave_lds_sync();
        const CoarsePool pl{C, (d + 15) / 16, 16, d, w, tile};
        pos = draw_slots(key, c0, c1, c2, E.k, carry,
                         [&pl](uint64_t r, int64_t& m, uint64_t& Sm, uint32_t& bm) {
                             coarse_search<true>(pl, r, m, Sm, bm);
                         },
                         ownp);
    }
    emit_slots(p, E, pos);
}

__global__ void __launch_bounds__(kBlock) k_select(SampleLayer p) {
    __shared__ uint32_t tiles[kWavesPerBlock][kTilePad];
    __shared__ uint64_t coarse[kWavesPerBlock][kWaveC + 1];
    __shared__ int32_t owners[kWavesPerBlock][kWaveMaxD];
    const int wid = uniform_i32(threadIdx.x / kWave);
    const int64_t fcount = p.ctl->fcount[p.layer];
    const int64_t out_base = p.ctl->out_base[p.layer];
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t e = blockIdx.x * (int64_t)kWavesPerBlock + wid; e < fcount; e += waves)
        select_entry(p, e, out_base, tiles[wid], coarse[wid], owners[wid]);
}

// One block per mid-size weighted list (kWaveMaxD < d <= kMidMaxD): the
// block's waves load the list's tiles in parallel into LDS (transposed layout,
// the whole list stays resident), one thread per 16-group sums it, a block
// scan builds the coarse prefix, and wave 0 draws the slots with every search
// served from LDS.
__global__ void __launch_bounds__(kMidThreads) k_select_mid(SampleLayer p, const int32_t* __restrict__ mids) {
    __shared__ uint32_t wt[kMidMaxD + kMidMaxD / 16];
    __shared__ uint64_t C[kMidMaxD / 16 + 1];
    const int tid = threadIdx.x;
    const int wid = uniform_i32(tid / kWave);
    const int lane = lane_id();
    const int64_t nm = (int64_t)p.ctl->nmid[p.layer];
    const int64_t out_base = p.ctl->out_base[p.layer];
    for (int64_t h = blockIdx.x; h < nm; h += gridDim.x) {
        EntryInfo E;
        load_entry(p, mids[h], out_base, E);
        const int64_t d = E.d;
        const uint32_t* w = (E.kind == kEdgeWeight ? p.g.ew : p.g.degw) + E.beg;
        for (int64_t t = wid; t * kTile < d; t += kMidWaves) {
            uint32_t x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int64_t idx = t * kTile + c * kWave + lane;
                x[c] = idx < d ? w[idx] : 0u;
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) wt[tpad((int)(t * kTile) + c * kWave + lane)] = x[c];
        }
        __syncthreads();
        const int ng = (int)((d + 15) / 16);
        // group sums, then inclusive scan of C[1..ng] (thread tid owns 2 groups)
        uint64_t s0 = 0, s1 = 0;
        const int g0 = 2 * tid, g1 = 2 * tid + 1;
        if (g0 < ng)
            for (int q = 0; q < 16; ++q) s0 += (16 * g0 + q < d) ? wt[tpad(16 * g0 + q)] : 0u;
        if (g1 < ng)
            for (int q = 0; q < 16; ++q) s1 += (16 * g1 + q < d) ? wt[tpad(16 * g1 + q)] : 0u;
        int64_t tot;
        const uint64_t before = (uint64_t)block_excl_scan_i64<kMidThreads>((int64_t)(s0 + s1), &tot);
        if (g0 < ng) C[g0 + 1] = before + s0;
        if (g1 < ng) C[g1 + 1] = before + s0 + s1;
        if (tid == 0) C[0] = 0;
        __syncthreads();
        if (wid == 0) {
            if (E.o + E.c > p.capacity) {
                if (lane == 0) p.ctl->overflow = 1;
            } else {
                const CoarsePool pl{C, ng, 16, d, w, wt};
                const int64_t pos = draw_slots(Key{p.k0, p.k1}, (uint32_t)(p.instance_base + (uint64_t)E.inst),
                                               (uint32_t)p.layer, (uint32_t)E.v, E.k, C[ng],
                                               [&pl](uint64_t r, int64_t& m, uint64_t& Sm, uint32_t& bm) {
                                                   coarse_search<true>(pl, r, m, Sm, bm);
                                               });
                emit_slots(p, E, pos);
            }
        }
        __syncthreads();
    }
}

// One block per hub list: the block's waves stream the list in tiles and add
// group sums into C (LDS atomics), a block scan turns them into the coarse
// prefix, then wave 0 draws the slots.
__global__ void __launch_bounds__(kHubThreads) k_select_hub(SampleLayer p, const int32_t* __restrict__ hubs) {
    __shared__ uint64_t C[kHubC + 1];
    __shared__ uint32_t tiles[kHubWaves][kTilePad];
    const int tid = threadIdx.x;
    const int wid = uniform_i32(tid / kWave);
    const int lane = lane_id();
    const int64_t nh = (int64_t)p.ctl->nhub[p.layer];
    const int64_t out_base = p.ctl->out_base[p.layer];
    for (int64_t h = blockIdx.x; h < nh; h += gridDim.x) {
        EntryInfo E;
        load_entry(p, hubs[h], out_base, E);
        const int64_t d = E.d;
        const uint32_t* w = (E.kind == kEdgeWeight ? p.g.ew : p.g.degw) + E.beg;
        int64_t g = 16;
        while ((d + g - 1) / g > kHubC) g <<= 1;
        const int64_t ng = (d + g - 1) / g;
        for (int64_t i = tid; i <= ng; i += kHubThreads) C[i] = 0;
        __syncthreads();
        for (int64_t t = wid; t * kTile < d; t += kHubWaves) {
            const uint64_t s = tile_group_sums(w, t * kTile, d, tiles[wid]);
            const int64_t first = t * kTile + lane * 16;
            if (first < d && s) atomicAdd((unsigned long long*)&C[1 + first / g], (unsigned long long)s);
        }
        __syncthreads();
        // inclusive scan of C[1..ng]; thread tid owns a contiguous segment
        const int64_t seg = (ng + kHubThreads - 1) / kHubThreads;
        const int64_t b0 = 1 + tid * seg;
        const int64_t b1 = (b0 + seg < ng + 1) ? b0 + seg : ng + 1;
        uint64_t local = 0;
        for (int64_t b = b0; b < b1; ++b) local += C[b];
        int64_t tot;
        uint64_t run = (uint64_t)block_excl_scan_i64<kHubThreads>((int64_t)local, &tot);
        for (int64_t b = b0; b < b1; ++b) {
            run += C[b];
            C[b] = run;
        }
        __syncthreads();
        if (wid == 0) {
            if (E.o + E.c > p.capacity) {
                if (lane == 0) p.ctl->overflow = 1;
            } else {
                const CoarsePool pl{C, ng, g, d, w, nullptr};
                const int64_t pos = draw_slots(Key{p.k0, p.k1}, (uint32_t)(p.instance_base + (uint64_t)E.inst),
                                               (uint32_t)p.layer, (uint32_t)E.v, E.k, C[ng],
                                               [&pl](uint64_t r, int64_t& m, uint64_t& Sm, uint32_t& bm) {
                                                   coarse_search<false>(pl, r, m, Sm, bm);
                                               });
                emit_slots(p, E, pos);
            }
        }
        __syncthreads();
    }
}

__global__ void k_segments(SampleLayer p, const int64_t* __restrict__ fstart, int64_t* __restrict__ offsets) {
    const int64_t fcount = p.ctl->fcount[p.layer];
    const int64_t total = p.ctl->total[p.layer];
    const int64_t base = p.ctl->out_base[p.layer];
    if (offsets) {
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p.num_instances;
             i += (int64_t)gridDim.x * blockDim.x) {
            const int64_t fs = fstart[i];
            offsets[(int64_t)p.layer * p.num_instances + i] = base + (fs < fcount ? p.off[fs] : total);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) p.ctl->out_base[p.layer + 1] = base + total;
}

__global__ void k_clear_visited(const int32_t* __restrict__ fv, const int32_t* __restrict__ fi,
                                const int64_t* __restrict__ fcount_p, uint32_t* __restrict__ visited,
                                int64_t nwp) {
    const int64_t fcount = *fcount_p;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < fcount;
         e += (int64_t)gridDim.x * blockDim.x)
        visited[(int64_t)fi[e] * nwp + (fv[e] >> 5)] = 0u;
}

}  // namespace

// ---------------------------------------------------------------- launchers
void launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, kBlock, 65536)), dim3(kBlock), 0, s, p, value, count);
}

void launch_degree_weights(const int64_t* rowptr, const int32_t* col, int64_t m, uint32_t* degw,
                           hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_degree_weights, dim3(grid_for(m, kBlock, 65536)), dim3(kBlock), 0, s, rowptr, col,
                       m, degw);
}

void launch_positive_counts(const int64_t* rowptr, const uint32_t* w, int64_t n, int32_t* ppos,
                            hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_positive_counts, dim3(grid_for(n, kWavesPerBlock, 65536)), dim3(kBlock), 0, s,
                       rowptr, w, n, ppos);
}

void launch_mark_seeds(const int32_t* seeds, int64_t num_seeds, const int64_t* seed_offsets, int32_t ni,
                       int64_t n, uint32_t* next, int64_t nwp, SampleCtl* ctl, hipStream_t s) {
    if (num_seeds <= 0) return;
    hipLaunchKernelGGL(k_mark_seeds, dim3(grid_for(num_seeds, kBlock, 65536)), dim3(kBlock), 0, s, seeds,
                       num_seeds, seed_offsets, ni, n, next, nwp, ctl);
}

void launch_bitmap_compact(uint32_t* next, uint32_t* visited, int64_t words, int64_t nwp,
                           int64_t* blocksum, int64_t* fcount_out, int32_t* fv, int32_t* fi,
                           int64_t* fstart, int32_t ni, hipStream_t s) {
    (void)ni;
    const int64_t n4 = words / 4;
    const int64_t nb = (n4 + kBlock - 1) / kBlock;
    if (nb <= 0) {
        launch_fill_u32((uint32_t*)fcount_out, 0u, 2, s);
        return;
    }
    hipLaunchKernelGGL(k_bm_count, dim3((unsigned)nb), dim3(kBlock), 0, s, (const uint4*)next, n4, blocksum);
    hipLaunchKernelGGL(k_scan_blocksums, dim3(1), dim3(1024), 0, s, blocksum, nb, (const int64_t*)nullptr,
                       (int64_t)1, fcount_out);
    hipLaunchKernelGGL(k_bm_emit, dim3((unsigned)nb), dim3(kBlock), 0, s, (uint4*)next, (uint4*)visited, n4,
                       nwp / 4, blocksum, fv, fi, fstart);
}

void launch_count(const SampleLayer& p, int32_t* cnt, int64_t cap_entries, hipStream_t s) {
    if (cap_entries <= 0) return;
    hipLaunchKernelGGL(k_count, dim3(grid_for(cap_entries, kBlock, 16384)), dim3(kBlock), 0, s, p, cnt);
}

void launch_scan_counts(const int32_t* cnt, const int64_t* fcount, int64_t cap_entries, int64_t* blocksum,
                        int64_t* off, int64_t* total_out, hipStream_t s) {
    const int64_t nb = (cap_entries + kScanItems - 1) / kScanItems;
    if (nb <= 0) {
        launch_fill_u32((uint32_t*)total_out, 0u, 2, s);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, cnt, fcount, blocksum);
    hipLaunchKernelGGL(k_scan_blocksums, dim3(1), dim3(1024), 0, s, blocksum, nb, fcount, (int64_t)kScanItems,
                       total_out);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, cnt, fcount, blocksum, off);
}

void launch_select(const SampleLayer& p, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(grid), dim3(kBlock), 0, s, p);
}

void launch_select_mid(const SampleLayer& p, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_select_mid, dim3(grid), dim3(kMidThreads), 0, s, p, (const int32_t*)p.mids);
}

void launch_select_hub(const SampleLayer& p, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_select_hub, dim3(grid), dim3(kHubThreads), 0, s, p, (const int32_t*)p.hubs);
}

void launch_segments(const SampleLayer& p, const int64_t* fstart, int64_t* offsets, hipStream_t s) {
    hipLaunchKernelGGL(k_segments, dim3(grid_for(p.num_instances, kBlock, 4096)), dim3(kBlock), 0, s, p,
                       fstart, offsets);
}

void launch_clear_visited(const int32_t* fv, const int32_t* fi, const int64_t* fcount, int64_t cap_entries,
                          uint32_t* visited, int64_t nwp, hipStream_t s) {
    if (cap_entries <= 0) return;
    hipLaunchKernelGGL(k_clear_visited, dim3(grid_for(cap_entries, kBlock, 16384)), dim3(kBlock), 0, s, fv,
                       fi, fcount, visited, nwp);
}

}  // namespace csaw
