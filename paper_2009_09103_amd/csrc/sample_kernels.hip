// sample_kernels.hip -- gfx950 kernels of neighbor sampling.
//
// One layer of the generic sampling loop (fig:api(b)) is
//   frontier build : next bitmap -> sorted frontier entries, each with its
//                    edge count min(k, P), edge offset, list fields and
//                    route (one pass with a decoupled look-back);
//                    visited |= next
//   select         : one wavefront per frontier vertex: EdgeBias, exact
//                    prefix, Philox draws, inverse transform search,
//                    collision rounds, direct draw from the updated prefix;
//                    writes the edges and marks new neighbors in the
//                    instance's next bitmap. Small entries are served by
//                    sub-wave groups (select_small); weighted lists longer
//                    than kWaveMaxD, or with a total weight of 2^32 or more,
//                    one wavefront each (select_big), searched through the
//                    graph's chunk prefix tables.
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

// ------------------------------------------------------------------ misc
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Edges of a batch to their requests' result arrays: segment j (edges
// [off[j], off[j+1]) of the batch's layer-major arrays, off non-decreasing)
// goes to to_src[j] and to_dst[j] (null: nowhere). A thread per edge finds
// its segment by binary search over off (a few hundred entries, cached), so
// a long segment is spread over the whole grid.
__global__ void k_scatter_segments(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                   const int64_t* __restrict__ off, int64_t nseg, int32_t* const* __restrict__ to_src,
                                   int32_t* const* __restrict__ to_dst) {
    const int64_t total = off[nseg];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = nseg;  // the last j with off[j] <= k
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (off[mid] <= k) lo = mid;
            else hi = mid;
        }
        int32_t* ts = to_src[lo];
        int32_t* td = to_dst[lo];
        if (!ts || !td) continue;
        ts[k - off[lo]] = src[k];
        td[k - off[lo]] = dst[k];
    }
}

__global__ void k_degree_weights(RowPtr rowptr, const int32_t* __restrict__ col,
                                 int64_t m, uint32_t* __restrict__ degw) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = col[e];
        degw[e] = (uint32_t)(rowptr[x + 1] - rowptr[x]);
    }
}

// one wavefront per vertex: number of positive weights in its list, with
// kWideList set when the list's total weight needs more than 32 bits, and
// the total itself
__global__ void k_positive_counts(RowPtr rowptr, const uint32_t* __restrict__ w,
                                  int64_t n, int32_t* __restrict__ ppos, uint64_t* __restrict__ wtot) {
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t v = blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave; v < n; v += waves) {
        const int64_t b = rowptr[v], e = rowptr[v + 1];
        int64_t c = 0;
        uint64_t tot = 0;
        for (int64_t i = b + lane; i < e; i += kWave) {
            c += (w[i] > 0);
            tot += w[i];
        }
        c = wave_sum_i64(c);
        tot = wave_sum_u64(tot);
        if (lane == 0) {
            ppos[v] = (int32_t)c | ((tot >> 32) ? kWideList : 0);
            wtot[v] = tot;
        }
    }
}

// ------------------------------------------------------------- frontier
// Seeds -> next bitmap of their instance (instance of seed s: the largest i
// with seed_offsets[i] <= s).
__global__ void k_mark_seeds(const int32_t* __restrict__ seeds, int64_t num_seeds,
                             const int64_t* __restrict__ seed_off, int32_t ni, int64_t n,
                             uint32_t* __restrict__ next, int64_t nwp, uint32_t* __restrict__ summ, int64_t nsw,
                             SampleCtl* ctl) {
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
        const uint32_t old = atomicOr(&next[(int64_t)lo * nwp + (v >> 5)], 1u << (v & 31));
        if (summ && old == 0u) atomicOr(&summ[(int64_t)lo * nsw + (v >> 10)], 1u << ((v >> 5) & 31));
    }
}

// ------------------------------------------------------------------ count
// Weighted lists that need draws are routed by length: up to kWaveMaxD
// candidates with a total weight below 2^32 to the wavefront kernel (list and
// 32-bit prefix resident in registers); the others to the long-list path,
// which draws with one wavefront per list from a coarse table built out of
// the graph's chunk prefix table (lists longer than kWaveMaxD; the table is
// computed once per graph and weight array, since it depends on the list
// alone, not on the instance) or, for shorter lists with a wide total, out of
// the list's one chunk reduced on the spot.

enum { kRouteWave = 0, kRouteBig = 1 };

__device__ __forceinline__ int route_of(int32_t kind, int32_t k, int32_t P, int64_t d, bool wide) {
    if (kind == kUniform || k <= 0 || k >= P || (d <= kWaveMaxD && !wide)) return kRouteWave;
    return kRouteBig;
}

// Forest fire NeighborSize (Section II-A): vertex v burns G neighbors, G
// geometric with P(G >= j) = (burn / 2^32)^j, capped at cap. Trial j
// succeeds iff word j mod 4 of the Philox block with counter
// (c0, c1, c2, kBurnRound << 16 | j / 4) is below burn.
__device__ __forceinline__ int32_t burn_count(Key key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t burn,
                                              int32_t cap) {
    int32_t g = 0;
    for (uint32_t blk = 0; g < cap; ++blk) {
        const uint4 x = philox4(key.k0, key.k1, c0, c1, c2, (kBurnRound << 16) | blk);
        const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (g >= cap || w[q] >= burn) return g;
            ++g;
        }
    }
    return g;
}

// NeighborSize of frontier vertex v of an instance with layer fanout k. The
// kernels that call it are instantiated with and without forest fire, so
// the burning code costs the fixed-fanout kernels no registers.
template <bool kBurn>
__device__ __forceinline__ int32_t neighbor_size(int32_t k, uint32_t burn, uint64_t key, uint32_t c0,
                                                 int32_t layer, int32_t v) {
    if (!kBurn || !burn || k == 0) return k;
    return burn_count(Key{(uint32_t)key, (uint32_t)(key >> 32)}, c0, (uint32_t)layer, (uint32_t)v, burn,
                      k < 0 ? kBurnCapAll : k);
}

// Positive biases of v's list with the kWideList flag (the list length if
// unbiased).
__device__ __forceinline__ int32_t positive_info(const GraphDev& g, int32_t kind, int32_t v, int64_t d) {
    if (kind == kUniform) return (int32_t)d;
    return kind == kEdgeWeight ? g.ppos_ew[v] : g.ppos_deg[v];
}

__device__ __forceinline__ int32_t entry_count(const GraphDev& g, int32_t k, int32_t kind, int32_t v,
                                               int32_t& route, int64_t& beg, int64_t& d, int32_t& pinfo,
                                               SampleCtl* ctl) {
    beg = g.rowptr[v];
    d = g.rowptr[v + 1] - beg;
    pinfo = positive_info(g, kind, v, d);
    const int32_t P = pinfo & ~kWideList;
    const bool wide = (pinfo & kWideList) != 0;
    route = kRouteWave;
    if (k == 0 || P == 0) return 0;
    if (k < 0 || k >= P) return P;
    if (k > kMaxDrawFanout) {
        ctl->unsupported = 1;
        return 0;
    }
    route = route_of(kind, k, P, d, wide);
    return k;
}

__device__ __forceinline__ int64_t chunks_of(int64_t d) { return (d + kChunk - 1) / kChunk; }

// Look-back status words: a 48-bit value, a valid bit and the build's epoch
// in one 64-bit word, so a reader never sees a value without its flag.
constexpr uint64_t kStatusValid = 1ull << 48;
constexpr uint64_t kStatusMask = kStatusValid - 1;
constexpr uint32_t kSpinLimit = 1u << 20;

__device__ __forceinline__ uint64_t status_pack(int64_t v, uint32_t epoch) {
    return ((uint64_t)v & kStatusMask) | kStatusValid | ((uint64_t)(epoch & 0x7FFF) << 49);
}
__device__ __forceinline__ bool status_ok(uint64_t w, uint32_t epoch) {
    return (w & kStatusValid) && (w >> 49) == (epoch & 0x7FFF);
}
__device__ __forceinline__ void status_store(unsigned long long* p, uint64_t v) {
    __hip_atomic_store(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t status_load(unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Next set bit of a word (cleared from it), or -1.
__device__ __forceinline__ int32_t pop_bit(uint32_t& bits) {
    if (!bits) return -1;
    const int32_t b = __ffs(bits) - 1;
    bits &= bits - 1;
    return b;
}

// Decoupled look-back of block b for two running totals (a, c), called by
// the 64 lanes of one wavefront: publishes b's aggregates, then sums its
// predecessors' published values 64 blocks at a time, nearest first; a
// predecessor's inclusive prefix ends the walk (blocks are dispatched in
// index order, so predecessors are resident or done). The spin is bounded and
// reports through *stuck instead of hanging. Publishes b's inclusive prefix
// and returns the exclusive ones (every lane).
__device__ __forceinline__ void lookback2(unsigned long long* status, int64_t b, int64_t tot_a, int64_t tot_c,
                                          uint32_t epoch, int32_t* stuck, int64_t& pa, int64_t& pc) {
    const int lane = lane_id();
    unsigned long long* st = status + 4 * b;
    if (b > 0 && lane == 0) {
        status_store(st + 0, status_pack(tot_a, epoch));
        status_store(st + 1, status_pack(tot_c, epoch));
    }
    pa = 0;
    pc = 0;
    int64_t end = b - 1;  // window covers predecessors end, end-1, ..., end-63
    uint32_t spins = 0;
    while (end >= 0) {
        const int64_t q = end - lane;
        int flag = 2;  // before block 0: an inclusive prefix of zero
        int64_t va = 0, vc = 0;
        if (q >= 0) {
            unsigned long long* sq = status + 4 * q;
            const uint64_t ia = status_load(sq + 2), ic = status_load(sq + 3);
            if (status_ok(ia, epoch) && status_ok(ic, epoch)) {
                va = (int64_t)(ia & kStatusMask);
                vc = (int64_t)(ic & kStatusMask);
            } else {
                const uint64_t aa = status_load(sq + 0), ac = status_load(sq + 1);
                if (status_ok(aa, epoch) && status_ok(ac, epoch)) {
                    flag = 1;
                    va = (int64_t)(aa & kStatusMask);
                    vc = (int64_t)(ac & kStatusMask);
                } else {
                    flag = 0;
                }
            }
        }
        const uint64_t incl = ballot(flag == 2);
        const uint64_t notready = ballot(flag == 0);
        const int first = incl ? __ffsll((unsigned long long)incl) - 1 : kWave;  // nearest inclusive
        const uint64_t upto = first >= kWave - 1 ? ~0ull : ((2ull << first) - 1);
        if (notready & upto) {  // a nearer predecessor has published nothing yet
            if (++spins > kSpinLimit) {  // never expected: report instead of hanging
                if (lane == 0) *stuck = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const bool take = ((upto >> lane) & 1ull) != 0;
        pa += (int64_t)wave_sum_u64(take ? (uint64_t)va : 0ull);
        pc += (int64_t)wave_sum_u64(take ? (uint64_t)vc : 0ull);
        if (first < kWave) break;
        end -= kWave;
        spins = 0;
    }
    if (lane == 0) {
        status_store(st + 2, status_pack(pa + tot_a, epoch));
        status_store(st + 3, status_pack(pc + tot_c, epoch));
    }
}

// Exclusive scans of four int64 per thread over the block in one pass (one
// pair of barriers); totals in tot[0..3]. Every thread must call it.
__device__ __forceinline__ void block_excl_scan4(int64_t (&x)[4], int64_t (&tot)[4]) {
    constexpr int kW = kBlock / kWave;
    __shared__ int64_t wsum[4][kW];
    const int lane = lane_id();
    const int wid = threadIdx.x / kWave;
    uint64_t incl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        incl[j] = wave_incl_scan_u64((uint64_t)x[j]);
        if (lane == kWave - 1) wsum[j][wid] = (int64_t)incl[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int64_t base = 0, t = 0;
#pragma unroll
        for (int w = 0; w < kW; ++w) {
            const int64_t v = wsum[j][w];
            if (w < wid) base += v;
            t += v;
        }
        tot[j] = t;
        x[j] = base + (int64_t)incl[j] - x[j];
    }
    __syncthreads();
}

// Frontier build of one layer, one pass: each thread takes G*V consecutive
// bitmap words (G loads of V words of next and of visited; small bitmaps use
// one word per thread for the most parallel blocks, large ones many, so that
// the number of blocks, each a short latency-bound chain of loads, stays
// small); it counts the new bits (entries), their edge counts min(k, P)
// (edges) and their long-list route (the words and the list fields are
// loaded again in the write pass rather than held in registers across the
// scan, which keeps occupancy up); a block scan plus a decoupled look-back
// over the blocks before it give global positions (blocks are dispatched in
// index order, so predecessors are resident or done; the spin is bounded and
// reports instead of hanging). The thread then writes its entries in
// (instance, vertex) order with count, edge offset, list fields and route,
// sets visited |= next, clears next, and the first word of an instance writes
// that instance's segment offset. The last block writes the layer's totals
// and the output base of the next layer.
template <int G, int V, bool kBurn, bool kSparse>
__global__ void __launch_bounds__(kBlock) k_frontier_build(FrontierBuild fb) {
    static_assert(V == 1 || V == 4, "one word or one 16-byte group per load");
    static_assert(!kSparse || (G == 1 && V == 1), "the dirty list gives one word per thread");
    __shared__ int64_t s_base_e, s_base_g;
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    // dense: every word of the bitmaps; sparse: the words of the dirty list
    // (grid sized by capacity, blocks past the list end at once)
    int64_t nwords = fb.nwords, nb = fb.nb;
    if (kSparse) {
        nwords = fb.ctl->ndirty[fb.layer];
        nb = nwords > 0 ? (nwords + kBlock - 1) / kBlock : 1;
        if (b >= nb) return;
    }
    const int64_t w0 = (b * kBlock + tid) * (G * V);  // first word of the thread (nwords is a multiple of 4)
    const int64_t wself = kSparse ? (w0 < nwords ? fb.dirty[w0] : 0) : w0;  // the thread's bitmap word
    const int64_t out_base = fb.ctl->out_base[fb.layer];
    uint32_t raws[G][V], viss[G][V];
    if (V == 4) {
        // next first; visited only where next has bits (large bitmaps are sparse)
        uint4 r4[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t iw = w0 + V * g;
            r4[g] = iw < fb.nwords ? *(const uint4*)(fb.next + iw) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t iw = w0 + V * g;
            const bool any = (r4[g].x | r4[g].y | r4[g].z | r4[g].w) != 0u;
            const uint4 v4 = any ? *(const uint4*)(fb.visited + iw) : make_uint4(0u, 0u, 0u, 0u);
            const uint32_t rr[4] = {r4[g].x, r4[g].y, r4[g].z, r4[g].w}, vv[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
            for (int q = 0; q < V; ++q) {
                raws[g][q] = rr[q];
                viss[g][q] = vv[q];
            }
        }
    }
    if (V == 1) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t iw = w0 + g, wd = kSparse ? wself : iw;
            raws[g][0] = iw < nwords ? fb.next[wd] : 0u;
            viss[g][0] = iw < nwords ? fb.visited[wd] : 0u;
        }
    }
    int64_t cnt4[4] = {0, 0, 0, 0};  // entries, edges, long lists, (unused)
    {
        int64_t inst_k = -1;
        int32_t k = 0, kind = 0;
        uint64_t key = 0;
        uint32_t iid = 0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const uint32_t w = raws[g][q] & ~viss[g][q];  // picks of visited vertices are not new
                if (!w) continue;
                const int64_t iw = kSparse ? wself : w0 + V * g + q;
                const int64_t inst = iw / fb.nwp;
                if (inst != inst_k) {
                    inst_k = inst;
                    k = fb.fanout[inst];
                    kind = fb.bias[inst];
                    if (kBurn) {
                        key = fb.inst_key[inst];
                        iid = fb.inst_id[inst];
                    }
                }
                const int32_t vbase = (int32_t)((iw - inst * fb.nwp) * 32);
                cnt4[0] += __popc(w);
                uint32_t bits = w;
                while (bits) {  // four bits at a time so that their loads overlap
                    int32_t bv[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) bv[t] = pop_bit(bits);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        int32_t route = kRouteWave, pinfo = 0;
                        int64_t beg = 0, d = 0;
                        int32_t c = 0;
                        if (bv[t] >= 0) {
                            const int32_t kv = neighbor_size<kBurn>(k, fb.burn, key, iid, fb.layer, vbase + bv[t]);
                            c = entry_count(fb.g, kv, kind, vbase + bv[t], route, beg, d, pinfo, fb.ctl);
                            cnt4[1] += c;
                            if (route == kRouteBig) ++cnt4[2];
                        }
                    }
                }
            }
        }
    }
    int64_t tot4[4];
    int64_t ex4[4] = {cnt4[0], cnt4[1], cnt4[2], cnt4[3]};
    block_excl_scan4(ex4, tot4);
    const int64_t ex_e = ex4[0], ex_g = ex4[1];
    int64_t ex_big = ex4[2];
    const int64_t tot_e = tot4[0], tot_g = tot4[1], tot_big = tot4[2];
    __shared__ int64_t s_big_base;
    if (tid == kWave) {  // wave 1: one reservation per block for its long lists
        s_big_base = tot_big ? (int64_t)atomicAdd(&fb.ctl->nbig[fb.layer], (unsigned long long)tot_big) : 0;
    }
    if (tid < kWave) {  // wave 0: publish, then look back 64 predecessors per step
        int64_t pe = 0, pg = 0;
        lookback2(fb.status, b, tot_e, tot_g, kSparse ? 2u * fb.layer + 2u : (uint32_t)fb.layer + 1u,
                  &fb.ctl->lookback_stuck, pe, pg);
        if (tid == 0) {
            s_base_e = pe;
            s_base_g = pg;
        }
    }
    __syncthreads();
    int64_t pos = s_base_e + ex_e;
    int64_t eoff = s_base_g + ex_g;
    int64_t inst_k = -1;
    int32_t k = 0, kind = 0;
    uint64_t key = 0;
    uint32_t iid = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (w0 + V * g >= nwords) break;
        const int64_t iw4 = kSparse ? wself : w0 + V * g;
        // the words again (L2): keeping them in registers across the scan
        // costs occupancy
        if (V == 4) {
            const uint4 r4 = *(const uint4*)(fb.next + iw4);
            const bool any = (r4.x | r4.y | r4.z | r4.w) != 0u;
            const uint4 v4 = any ? *(const uint4*)(fb.visited + iw4) : make_uint4(0u, 0u, 0u, 0u);
            const uint32_t rr[4] = {r4.x, r4.y, r4.z, r4.w}, vv[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
            for (int q = 0; q < V; ++q) {
                raws[g][q] = rr[q];
                viss[g][q] = vv[q];
            }
        } else {
            raws[g][0] = fb.next[iw4];
            viss[g][0] = fb.visited[iw4];
        }
        uint32_t newv[V];
        bool any_raw = false, any_new = false;
#pragma unroll
        for (int q = 0; q < V; ++q) {
            const int64_t iw = iw4 + q;
            const uint32_t w = raws[g][q] & ~viss[g][q];
            newv[q] = viss[g][q] | w;
            any_raw |= raws[g][q] != 0u;
            any_new |= w != 0u;
            const int64_t inst = iw / fb.nwp;
            const int64_t local = iw - inst * fb.nwp;
            if (fb.offsets && fb.layer < fb.num_layers) {
                if (!kSparse) {
                    if (local == 0) fb.offsets[(int64_t)fb.layer * fb.num_instances + inst] = out_base + eoff;
                } else {
                    // the first dirty word of an instance starts its segment, and
                    // those of the instances since the previous dirty word's (empty)
                    const int64_t prev = w0 > 0 ? fb.dirty[w0 - 1] / fb.nwp : -1;
                    for (int64_t i = prev + 1; i <= inst; ++i)
                        fb.offsets[(int64_t)fb.layer * fb.num_instances + i] = out_base + eoff;
                }
            }
            if (!w) continue;
            if (inst != inst_k) {
                inst_k = inst;
                k = fb.fanout[inst];
                kind = fb.bias[inst];
                if (kBurn) {
                    key = fb.inst_key[inst];
                    iid = fb.inst_id[inst];
                }
            }
            const int32_t vbase = (int32_t)(local * 32);
            uint32_t bits = w;
            while (bits) {
                int32_t bv[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) bv[t] = pop_bit(bits);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (bv[t] < 0) continue;
                    const int32_t v = vbase + bv[t];
                    int32_t route, c, pinfo;
                    int64_t beg, d;
                    c = entry_count(fb.g, neighbor_size<kBurn>(k, fb.burn, key, iid, fb.layer, v), kind, v, route, beg, d,
                                    pinfo, fb.ctl);
                    fb.fv[pos] = v;
                    fb.fi[pos] = (int32_t)inst;
                    fb.cnt[pos] = c;
                    fb.off[pos] = eoff;
                    fb.fbeg[pos] = beg;
                    fb.fdeg[pos] = (int32_t)d;
                    fb.fpos[pos] = pinfo;
                    if (route == kRouteBig) fb.bigs[s_big_base + ex_big++] = (int32_t)pos;
                    ++pos;
                    eoff += c;
                }
            }
        }
        if (V == 4) {
            if (any_new) *(uint4*)(fb.visited + iw4) = make_uint4(newv[0], newv[V > 1 ? 1 : 0], newv[V > 2 ? 2 : 0],
                                                                  newv[V > 3 ? 3 : 0]);
            if (any_raw) *(uint4*)(fb.next + iw4) = make_uint4(0u, 0u, 0u, 0u);  // also words that held only visited picks
        } else {
            if (any_new) fb.visited[iw4] = newv[0];
            if (any_raw) fb.next[iw4] = 0u;
        }
    }
    if (b == nb - 1) {  // last block: totals, and the bases of the layers after this one
        const int64_t te = s_base_e + tot_e, tg = s_base_g + tot_g;
        const int64_t ob = out_base + tg;
        if (tid == 0) {
            fb.ctl->fcount[fb.layer] = te;
            fb.ctl->total[fb.layer] = tg;
            for (int j = fb.layer + 1; j <= fb.num_layers; ++j) fb.ctl->out_base[j] = ob;
        }
        if (fb.offsets) {
            const int64_t ni = fb.num_instances;
            const int64_t first_l = fb.nwp > 0 ? fb.layer + 1 : fb.layer;
            for (int64_t j = first_l; j < fb.num_layers; ++j)
                for (int64_t i = tid; i < ni; i += kBlock) fb.offsets[j * ni + i] = (j == fb.layer ? out_base : ob);
            if (tid == 0) fb.offsets[(int64_t)fb.num_layers * ni] = ob;
            if (kSparse && fb.layer < fb.num_layers) {  // instances after the last dirty word's: empty at the end
                const int64_t last = nwords > 0 ? fb.dirty[nwords - 1] / fb.nwp : -1;
                for (int64_t i = last + 1 + tid; i < ni; i += kBlock) fb.offsets[(int64_t)fb.layer * ni + i] = ob;
            }
        }
    }
}

// Sparse frontier build, first pass: the summary bitmap (one bit per word of
// the instances' next bitmaps, set by the claim that made the word non-zero)
// is compacted into the list of dirty words, in increasing order, with a
// decoupled look-back over the blocks; the summary is cleared as it is read.
// Each thread takes four summary words (the summary of an instance is a
// multiple of four words).
__global__ void __launch_bounds__(kBlock) k_dirty_compact(FrontierBuild fb) {
    __shared__ int64_t s_base;
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t nsumm = (int64_t)fb.num_instances * fb.nsw;
    const int64_t i0 = (b * kBlock + tid) * 4;
    const uint4 s4 = i0 < nsumm ? *(const uint4*)(fb.summ + i0) : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t sw[4] = {s4.x, s4.y, s4.z, s4.w};
    int64_t cnt4[4] = {(int64_t)(__popc(sw[0]) + __popc(sw[1]) + __popc(sw[2]) + __popc(sw[3])), 0, 0, 0};
    int64_t tot4[4];
    block_excl_scan4(cnt4, tot4);
    if (tid < kWave) {
        int64_t pa = 0, pc = 0;
        lookback2(fb.status, b, tot4[0], 0, 2u * fb.layer + 1u, &fb.ctl->lookback_stuck, pa, pc);
        if (tid == 0) s_base = pa;
    }
    __syncthreads();
    int64_t pos = s_base + cnt4[0];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t i = i0 + q;
        const int64_t inst = i / fb.nsw;
        const int64_t wbase = inst * fb.nwp + (i - inst * fb.nsw) * 32;
        for (uint32_t bits = sw[q]; bits; bits &= bits - 1) fb.dirty[pos++] = wbase + (__ffs(bits) - 1);
    }
    if ((s4.x | s4.y | s4.z | s4.w) != 0u) *(uint4*)(fb.summ + i0) = make_uint4(0u, 0u, 0u, 0u);
    if (b == fb.nb_dirty - 1 && tid == 0) fb.ctl->ndirty[fb.layer] = s_base + tot4[0];
}

// ----------------------------------------------------------------- select
// Lists of the wavefront kernel (weighted d <= kWaveMaxD, and every unbiased
// list) are searched in registers (draw_resident) or directly (r is the
// position for unbiased lists). Long lists use a coarse table: groups of
// g = 16 consecutive candidates, C[t] = S[t*g] (exclusive prefix at the group
// starts) and C[nc] = W in LDS; a search finds the group by binary search in
// C and the candidate by scanning the group's weights from global memory / L2.
//
// Chunk reduction stages weights through LDS in tiles of 1024: 16 coalesced
// loads per lane are issued together, stored transposed (element i at
// i + i/16, so that lane L's 16 consecutive elements sit in 16 distinct
// banks) and summed per lane.
constexpr int kTile = 1024;
constexpr int kTilePad = kTile + kTile / 16;

__device__ __forceinline__ int tpad(int i) { return i + (i >> 4); }

struct CoarsePool {
    const uint64_t* C;      // LDS, nc + 1 entries
    int64_t nc;             // groups
    int64_t g;              // group length
    int64_t d;              // list length
    const uint32_t* w;      // weights of the list in global memory
};

// Scan weights w[i..end) from global memory, 16 loads in flight, for the
// first candidate whose running total (from acc) exceeds r: running totals
// are monotone, so its index in a batch is the number of totals <= r.
__device__ __forceinline__ void fine_scan_global(const uint32_t* __restrict__ w, int64_t i, int64_t end,
                                                 uint64_t acc, uint64_t r, int64_t& m, uint64_t& Sm,
                                                 uint32_t& bm) {
    m = i;
    Sm = acc;
    bm = 0;
    for (; i < end; i += 16) {
        const uint32_t* wp = w + i;
        const int n = end - i < 16 ? (int)(end - i) : 16;
        uint32_t x[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) x[q] = q < n ? wp[q] : 0u;
        int cnt = 0;
        uint64_t run = acc, before = acc;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            run += x[q];
            const bool le = run <= r;
            cnt += le;
            before = le ? run : before;
        }
        if (cnt < n) {
            m = i + cnt;
            Sm = before;
            bm = wp[cnt];
            return;
        }
        acc = run;
    }
}

// m = max{i in [0,d) : S_i <= r} with S_m and b_m; per lane: binary search
// for the group in the LDS table C, then the group's weights from global
// memory / L2.
__device__ __forceinline__ void coarse_search(const CoarsePool& pl, uint64_t r, int64_t& m, uint64_t& Sm,
                                              uint32_t& bm) {
    int64_t lo = 0, hi = pl.nc;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (pl.C[mid] <= r) lo = mid;
        else hi = mid;
    }
    const int64_t i = lo * pl.g;
    const int64_t end = (i + pl.g < pl.d) ? i + pl.g : pl.d;
    fine_scan_global(pl.w, i, end, pl.C[lo], r, m, Sm, bm);
}

// Draw k distinct candidates with one lane per slot (lane j = slot j < k) and
// a per-lane inverse transform search(r, m, Sm, bm). Each round every open
// slot draws; taken in slot order, a slot keeps its candidate unless it is
// already held -- which also covers a lower slot that took the same candidate
// in this round, so the lowest slot wins. Slots still open after `rounds` take
// direct draws from the prefix without the held candidates, in slot order:
// r0 in [0, W - held mass), mapped by the skip map (every held candidate whose
// start in the updated prefix is at or below r0 adds its bias) and searched
// with search_all (same r on every lane).
template <class Search, class SearchAll>
__device__ __forceinline__ int64_t draw_slots(Key key, uint32_t c0, uint32_t c1, uint32_t c2, int32_t k, int32_t rounds,
                                              uint64_t W, const Search& search, const SearchAll& search_all) {
    const int lane = lane_id();
    bool held = false;
    int64_t pos = 0;
    uint64_t Spos = 0;
    uint32_t bpos = 0;
    uint64_t open = k >= kWave ? ~0ull : ((1ull << k) - 1);
    for (int a = 0; a < rounds && open; ++a) {
        int64_t m = -1;
        uint64_t Sm = 0;
        uint32_t bm = 0;
        if ((open >> lane) & 1ull) search(draw(key, c0, c1, c2, (uint32_t)lane | ((uint32_t)a << 16), W), m, Sm, bm);
        for (uint64_t todo = open; todo; todo &= todo - 1) {
            const int j = __ffsll((unsigned long long)todo) - 1;
            const int64_t mj = readlane_i64(m, j);
            if (ballot(held && pos == mj) == 0) {
                if (lane == j) {
                    held = true;
                    pos = m;
                    Spos = Sm;
                    bpos = bm;
                }
                open &= ~(1ull << j);
            }
        }
    }
    if (open) {
        const uint64_t heldmask = ballot(held);
        // before = total bias of held candidates at smaller positions
        uint64_t before = 0;
        for (uint64_t hm = heldmask; hm; hm &= hm - 1) {
            const int q = __ffsll((unsigned long long)hm) - 1;
            const int64_t pq = readlane_i64(pos, q);
            const uint32_t bq = readlane_u32(bpos, q);
            if (held && pq < pos) before += bq;
        }
        uint64_t removed = wave_sum_u64(held ? (uint64_t)bpos : 0ull);
        for (; open; open &= open - 1) {
            const int j = __ffsll((unsigned long long)open) - 1;
            const uint64_t r0 = draw(key, c0, c1, c2, (uint32_t)j | (kFallbackRound << 16), W - removed);
            const uint64_t r = r0 + wave_sum_u64((held && Spos - before <= r0) ? (uint64_t)bpos : 0ull);
            int64_t m = 0;
            uint64_t Sm = 0;
            uint32_t bm = 0;
            search_all(r, m, Sm, bm);  // same r on every lane
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
        }
    }
    return pos;
}

// Weighted lists of at most 64*E candidates, resident in registers: lane L
// holds candidates [L*E, L*E+E) and their inclusive prefix S (width T; the
// wavefront route sends only lists with W < 2^32, so T = 32 bits there). A draw r is resolved by the whole wavefront: the
// owning lane is the number of lanes whose last prefix is <= r, the position
// inside it the number of its prefixes <= r. Held candidates are one bit per
// element in the owning lane. Slots are taken in slot order within a round,
// as in draw_slots; direct draws rescan the prefix with held weights removed,
// which is the updated prefix whose inverse the skip map computes.
template <int E, typename T>
__device__ __forceinline__ int32_t find_resident(const T (&S)[E], T r) {
    const int L = __popcll(ballot(S[E - 1] <= r));
    if (E == 1) return L;
    int32_t cl = 0;
#pragma unroll
    for (int e = 0; e < E - 1; ++e) cl += S[e] <= r ? 1 : 0;
    return L * E + readlane_i32(cl, L);
}

template <int E, typename T>
__device__ __forceinline__ int32_t draw_resident_t(const uint32_t (&x)[E], T excl, T W, Key key, uint32_t c0,
                                                   uint32_t c1, uint32_t c2, int32_t k, int32_t rounds) {
    const int lane = lane_id();
    T S[E];
    {
        T acc = excl;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            acc += (T)x[e];
            S[e] = acc;
        }
    }
    uint32_t hb = 0;  // held bits of this lane's candidates
    int32_t pos = 0;
    uint64_t open = k >= kWave ? ~0ull : ((1ull << k) - 1);
    for (int a = 0; a < rounds && open; ++a) {
        T rl = 0;
        if ((open >> lane) & 1ull) rl = (T)draw(key, c0, c1, c2, (uint32_t)lane | ((uint32_t)a << 16), (uint64_t)W);
        for (uint64_t todo = open; todo; todo &= todo - 1) {
            const int j = __ffsll((unsigned long long)todo) - 1;
            const int32_t m = find_resident<E, T>(S, readlane_t(rl, j));
            const int owner = m / E, bit = m % E;
            if (((readlane_u32(hb, owner) >> bit) & 1u) == 0) {
                if (lane == owner) hb |= 1u << bit;
                if (lane == j) pos = m;
                open &= ~(1ull << j);
            }
        }
    }
    if (open) {
        uint64_t u = 0;
        if ((open >> lane) & 1ull) u = philox_u64(key.k0, key.k1, c0, c1, c2, (uint32_t)lane | (kFallbackRound << 16));
        for (; open; open &= open - 1) {
            const int j = __ffsll((unsigned long long)open) - 1;
            T Sp[E];
            T ls = 0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                ls += ((hb >> e) & 1u) ? (T)0 : (T)x[e];
                Sp[e] = ls;
            }
            const T incl = wave_incl_scan_t(ls);
            const T ex = incl - ls;
#pragma unroll
            for (int e = 0; e < E; ++e) Sp[e] += ex;
            const T Wp = readlane_t(incl, kWave - 1);
            const T r0 = (T)range_reduce(readlane_u64(u, j), (uint64_t)Wp);
            const int32_t m = find_resident<E, T>(Sp, r0);
            if (lane == m / E) hb |= 1u << (m % E);
            if (lane == j) pos = m;
        }
    }
    return pos;
}

template <int E>
__device__ __forceinline__ int32_t draw_resident(const uint32_t* __restrict__ w, int64_t d, Key key, uint32_t c0,
                                                 uint32_t c1, uint32_t c2, int32_t k, int32_t rounds) {
    const int lane = lane_id();
    // d <= kWaveMaxD: 32-bit indices; every load is issued (clamped into the
    // list) and the tail zeroed after, so no lane branches
    const int32_t last = (int32_t)d - 1;
    uint32_t x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = w[min(lane * E + e, last)];
    uint32_t ls = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        x[e] = lane * E + e <= last ? x[e] : 0u;
        ls += x[e];
    }
    // routing guarantees W < 2^32, so every prefix fits 32 bits
    const uint32_t incl = wave_incl_scan_u32((uint32_t)ls);
    const uint32_t W = readlane_u32(incl, kWave - 1);
    return draw_resident_t<E, uint32_t>(x, incl - (uint32_t)ls, W, key, c0, c1, c2, k, rounds);
}

// A picked neighbor joins the instance's next bitmap unless it is visited or
// already there: picks concentrate on hubs, and skipping those atomics keeps
// them from queueing on a few hot words. (The frontier build also masks
// visited vertices.)
__device__ __forceinline__ void claim(bool do_claim, const uint32_t* visb, uint32_t* nextb, uint32_t* summb,
                                      int32_t x) {
    if (!do_claim) return;
    const uint32_t bit = 1u << (x & 31);
    const int64_t wd = x >> 5;
    if (!((visb[wd] | nextb[wd]) & bit)) {
        // the claim that makes a word non-zero records it in the summary (sparse builds)
        const uint32_t old = atomicOr(&nextb[wd], bit);
        if (summb && old == 0u) atomicOr(&summb[wd >> 5], 1u << (wd & 31));
    }
}

// The instance's summary bitmap (sparse builds) or null.
__device__ __forceinline__ uint32_t* summary_of(const SampleLayer& p, int64_t inst) {
    return p.summ ? p.summ + inst * p.nsw : nullptr;
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
    bool do_claim, wide;
    uint64_t key;
    uint32_t c0;
};

// A run of up to 64 consecutive frontier entries, one per lane: the entry's
// fields are read coalesced, then its instance's tables, so a wavefront pays
// two memory round trips for the whole run instead of several per entry.
struct EntryRun {
    int32_t c, v, inst, pinfo, k, kind, do_claim, c0;
    int32_t d;
    int64_t o, beg;
    uint64_t key;
};

template <bool kBurn>
__device__ __forceinline__ void load_run(const SampleLayer& p, int64_t e, bool valid, int64_t out_base,
                                         EntryRun& R) {
    R.c = valid ? p.cnt[e] : 0;
    R.v = valid ? p.fv[e] : 0;
    R.inst = valid ? p.fi[e] : 0;
    R.o = valid ? out_base + p.off[e] : 0;
    R.beg = valid ? p.fbeg[e] : 0;
    R.d = valid ? p.fdeg[e] : 0;
    R.pinfo = valid ? p.fpos[e] : 0;
    if (R.v < p.vlo || R.v >= p.vhi) R.c = 0;  // another partition's entry (out-of-memory schedule)
    R.k = R.kind = R.do_claim = 0;
    R.c0 = 0;
    R.key = 0;
    if (R.c) {
        R.k = p.fanout[R.inst];
        R.kind = p.bias[R.inst];
        R.do_claim = p.fanout_next[R.inst] != 0;
        R.key = p.inst_key[R.inst];
        R.c0 = p.inst_id[R.inst];
        R.k = neighbor_size<kBurn>(R.k, p.burn, R.key, (uint32_t)R.c0, p.layer, R.v);
    }
}

// A run kept in LDS (one array per field), so that its fields need no
// registers while the wavefront works through the run.
struct RunLds {
    int32_t c[kWave], v[kWave], inst[kWave], pinfo[kWave], k[kWave], kind[kWave], do_claim[kWave], c0[kWave],
        d[kWave];
    int64_t o[kWave], beg[kWave];
    uint64_t key[kWave];
};

__device__ __forceinline__ void store_run(RunLds& L, const EntryRun& R, int lane) {
    L.c[lane] = R.c;
    L.v[lane] = R.v;
    L.inst[lane] = R.inst;
    L.pinfo[lane] = R.pinfo;
    L.k[lane] = R.k;
    L.kind[lane] = R.kind;
    L.do_claim[lane] = R.do_claim;
    L.c0[lane] = R.c0;
    L.d[lane] = R.d;
    L.o[lane] = R.o;
    L.beg[lane] = R.beg;
    L.key[lane] = R.key;
}

// The fields of run entry j, wave-uniform.
__device__ __forceinline__ EntryInfo lds_entry(const RunLds& L, int j) {
    EntryInfo E;
    E.c = uniform_i32(L.c[j]);
    E.v = uniform_i32(L.v[j]);
    E.inst = uniform_i32(L.inst[j]);
    E.o = uniform_i64(L.o[j]);
    E.beg = uniform_i64(L.beg[j]);
    E.d = uniform_i32(L.d[j]);
    const int32_t pinfo = uniform_i32(L.pinfo[j]);
    E.P = pinfo & ~kWideList;
    E.wide = (pinfo & kWideList) != 0;
    E.k = uniform_i32(L.k[j]);
    E.kind = uniform_i32(L.kind[j]);
    E.do_claim = uniform_i32(L.do_claim[j]) != 0;
    E.key = (uint64_t)uniform_i64((int64_t)L.key[j]);
    E.c0 = (uint32_t)uniform_i32(L.c0[j]);
    return E;
}

// The fields of run entry j, wave-uniform.
__device__ __forceinline__ EntryInfo run_entry(const EntryRun& R, int j) {
    EntryInfo E;
    E.c = readlane_i32(R.c, j);
    E.v = readlane_i32(R.v, j);
    E.inst = readlane_i32(R.inst, j);
    E.o = readlane_i64(R.o, j);
    E.beg = readlane_i64(R.beg, j);
    E.d = readlane_i32(R.d, j);
    const int32_t pinfo = readlane_i32(R.pinfo, j);
    E.P = pinfo & ~kWideList;
    E.wide = (pinfo & kWideList) != 0;
    E.k = readlane_i32(R.k, j);
    E.kind = readlane_i32(R.kind, j);
    E.do_claim = readlane_i32(R.do_claim, j) != 0;
    E.key = readlane_u64(R.key, j);
    E.c0 = readlane_u32(R.c0, j);
    return E;
}

__device__ __forceinline__ void emit_slots(const SampleLayer& p, const EntryInfo& E, int64_t pos) {
    const int lane = lane_id();
    if (lane < E.k) {
        const int32_t x = p.g.col[E.beg + pos];
        p.src[E.o + lane] = E.v;
        p.dst[E.o + lane] = x;
        claim(E.do_claim, p.visited + (int64_t)E.inst * p.nwp, p.next + (int64_t)E.inst * p.nwp, summary_of(p, E.inst),
              x);
    }
}

__device__ void select_entry(const SampleLayer& p, const EntryInfo& E) {
    const int lane = lane_id();
    if (E.c == 0) return;
    if (E.o + E.c > p.capacity) {
        if (lane == 0) p.ctl->overflow = 1;
        return;
    }
    if (route_of(E.kind, E.k, E.P, E.d, E.wide) != kRouteWave) return;  // long-list path
    const uint32_t* visb = p.visited + (int64_t)E.inst * p.nwp;
    uint32_t* nextb = p.next + (int64_t)E.inst * p.nwp;
    uint32_t* summb = summary_of(p, E.inst);
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
                claim(E.do_claim, visb, nextb, summb, x);
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
                        claim(E.do_claim, visb, nextb, summb, nb);
                    }
                    run += __popcll(mask);
                }
            }
        }
        return;
    }

    // ---- k < P <= d: draw k distinct candidates (k <= kMaxDrawFanout)
    const Key key{(uint32_t)E.key, (uint32_t)(E.key >> 32)};
    const uint32_t c0 = E.c0;
    const uint32_t c1 = (uint32_t)p.layer;
    const uint32_t c2 = (uint32_t)E.v;
    int64_t pos;
    if (!weighted) {
        const auto pick = [](uint64_t r, int64_t& m, uint64_t& Sm, uint32_t& bm) {
            m = (int64_t)r;
            Sm = r;
            bm = 1;
        };
        pos = draw_slots(key, c0, c1, c2, E.k, p.rounds, (uint64_t)d, pick, pick);
    } else if (d <= 64) {
        pos = draw_resident<1>(w, d, key, c0, c1, c2, E.k, p.rounds);
    } else if (d <= 128) {
        pos = draw_resident<2>(w, d, key, c0, c1, c2, E.k, p.rounds);
    } else if (d <= 256) {
        pos = draw_resident<4>(w, d, key, c0, c1, c2, E.k, p.rounds);
    } else {
        pos = draw_resident<8>(w, d, key, c0, c1, c2, E.k, p.rounds);
    }
    emit_slots(p, E, pos);
}

// ------------------------------------------------------- sub-wave groups
// Entries whose work fits G lanes -- a take-all list of at most G
// candidates, an unbiased draw of at most G slots, a weighted draw from at
// most G candidates -- are served 64/G side by side, G lanes each: slot j of
// an entry is lane j of its group, a weighted candidate i is lane i. The
// rounds take each group's slots in slot order exactly as the full-wave path
// does (one slot index t at a time for all groups), so results do not depend
// on the grouping. An entry with slots still open after the rounds is returned
// to the full-wave path, which repeats its rounds and ends with direct draws.
// The bucket bounds (largest size served by 16- and 32-lane groups) are call
// parameters, so a tuner can pick them per workload.

// The value of x at lane (group base + t), on every lane of the group.
template <int G>
__device__ __forceinline__ uint32_t group_bcast_u32(uint32_t x, int t) {
    const int lane = lane_id();
    uint32_t r = readlane_u32(x, t);
#pragma unroll
    for (int q = 1; q < kWave / G; ++q) {
        const uint32_t y = readlane_u32(x, q * G + t);
        r = lane >= q * G ? y : r;
    }
    return r;
}

// Inclusive scan inside each group of G lanes (every lane active).
template <int G>
__device__ __forceinline__ uint32_t group_incl_scan_u32(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr1, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr2, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr4, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr8, 0xf, 0xf, false);
    if (G >= 32) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowBcast15, 0xa, 0xf, false);
    return x;
}

// Does run entry R (this lane's) fit groups of G lanes with bucket bound b?
__device__ __forceinline__ bool group_fits(const EntryRun& R, int64_t capacity, int32_t b) {
    if (R.c == 0 || R.o + R.c > capacity) return false;
    const int32_t P = R.pinfo & ~kWideList;
    if (route_of(R.kind, R.k, P, R.d, (R.pinfo & kWideList) != 0) != kRouteWave) return false;
    const bool take = R.k < 0 || R.k >= P;
    return (take || R.kind != kUniform) ? R.d <= b : R.k <= b;
}

template <int G>
__device__ uint64_t select_groups(const SampleLayer& p, const RunLds& R, uint64_t elig) {
    constexpr uint64_t kLow = (1ull << G) - 1;
    const int lane = lane_id();
    const int gl = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const uint64_t gmask = kLow << gbase;
    uint64_t back = 0;
    for (uint64_t rem = elig; rem;) {
        // the next 64/G eligible entries, one per group
        int srcl = -1;
#pragma unroll
        for (int q = 0; q < kWave / G; ++q) {
            const int s = rem ? __ffsll((unsigned long long)rem) - 1 : -1;
            rem = rem ? rem & (rem - 1) : 0ull;
            srcl = gbase == q * G ? s : srcl;
        }
        const bool valid = srcl >= 0;
        const int sl = valid ? srcl : 0;
        const int32_t v = R.v[sl];
        const int32_t inst = R.inst[sl];
        const int64_t o = R.o[sl];
        const int64_t beg = R.beg[sl];
        const int32_t d = R.d[sl];
        const int32_t P = R.pinfo[sl] & ~kWideList;
        const int32_t k = R.k[sl];
        const int32_t kind = R.kind[sl];
        const bool do_claim = R.do_claim[sl] != 0;
        const uint64_t ekey = R.key[sl];
        const uint32_t c0 = (uint32_t)R.c0[sl];
        const bool take = k < 0 || k >= P;
        const bool weighted = kind != kUniform;
        const uint32_t* w = (kind == kEdgeWeight ? p.g.ew : p.g.degw) + beg;  // read only if weighted

        // weights of a weighted group, one candidate per lane
        const bool wlist = valid && weighted && !(take && P == d);
        uint32_t x = 0;
        if (wlist && gl < d) x = w[gl];

        // take-all groups: every positive candidate, list order
        int32_t pos = -1, slot = gl;
        const uint64_t posm = ballot(valid && take && wlist && x > 0);
        if (valid && take && gl < d) {
            if (!wlist) pos = gl;
            else if (x > 0) {
                pos = gl;
                slot = __popcll(posm & gmask & lanemask_lt());
            }
        }

        // draw groups: rounds in slot order per group
        const bool drw = valid && !take;
        const uint32_t S = group_incl_scan_u32<G>(drw ? x : 0u);
        const uint32_t Wg = group_bcast_u32<G>(S, G - 1);
        const uint64_t W = weighted ? (uint64_t)Wg : (uint64_t)(uint32_t)d;
        const Key key{(uint32_t)ekey, (uint32_t)(ekey >> 32)};
        uint64_t open = ballot(drw && gl < k);
        int32_t hid = -1;  // candidate this lane marks held (uniform: its slot's pick; weighted: itself)
        for (int a = 0; a < p.rounds && open; ++a) {
            uint32_t r = 0;
            if ((open >> lane) & 1ull) r = (uint32_t)draw(key, c0, (uint32_t)p.layer, (uint32_t)v, (uint32_t)gl | ((uint32_t)a << 16), W);
            uint64_t tm = 0;
#pragma unroll
            for (int q = 0; q < kWave / G; ++q) tm |= (open >> (q * G)) & kLow;
            for (; tm; tm &= tm - 1) {
                const int t = __ffsll((unsigned long long)tm) - 1;
                const uint32_t rt = group_bcast_u32<G>(r, t);
                const int32_t mt = weighted ? __popcll(ballot(S <= rt) & gmask) : (int32_t)rt;
                const bool free = (ballot(hid >= 0 && hid == mt) & gmask) == 0;
                const bool acc = free && ((open >> (gbase + t)) & 1ull);
                if (acc) {
                    if (gl == t) pos = mt;
                    if (weighted ? gl == mt : gl == t) hid = mt;
                }
                open &= ~ballot(acc && gl == t);
            }
        }
        // groups with open slots go back to the full-wave path, unwritten
        const bool unfinished = (open & gmask) != 0;
        for (uint64_t ub = ballot(unfinished && gl == 0); ub; ub &= ub - 1)
            back |= 1ull << readlane_i32(sl, __ffsll((unsigned long long)ub) - 1);
        if (pos >= 0 && !unfinished) {
            const int32_t nb = p.g.col[beg + pos];
            p.src[o + slot] = v;
            p.dst[o + slot] = nb;
            claim(do_claim, p.visited + (int64_t)inst * p.nwp, p.next + (int64_t)inst * p.nwp, summary_of(p, inst), nb);
        }
    }
    return back;
}

// A sub-wave entry whose slots were still open after the rounds, redone by
// the whole wavefront: an unbiased draw of at most 32 slots or a weighted
// draw from at most 32 candidates (the draw branch of select_entry).
__device__ void select_entry_small_draw(const SampleLayer& p, const EntryInfo& E) {
    const Key key{(uint32_t)E.key, (uint32_t)(E.key >> 32)};
    const uint32_t c1 = (uint32_t)p.layer;
    const uint32_t c2 = (uint32_t)E.v;
    int64_t pos;
    if (E.kind == kUniform) {
        const auto pick = [](uint64_t r, int64_t& m, uint64_t& Sm, uint32_t& bm) {
            m = (int64_t)r;
            Sm = r;
            bm = 1;
        };
        pos = draw_slots(key, E.c0, c1, c2, E.k, p.rounds, (uint64_t)E.d, pick, pick);
    } else {
        pos = draw_resident<1>((E.kind == kEdgeWeight ? p.g.ew : p.g.degw) + E.beg, E.d, key, E.c0, c1, c2, E.k,
                                 p.rounds);
    }
    emit_slots(p, E, pos);
}

// Sub-wave entries of the layer: each wavefront takes runs of 64 frontier
// entries (grid-stride), keeps the run in LDS and serves its small entries
// in groups of 16 and 32 lanes; the other entries are left to k_select.
template <bool kBurn>
__global__ void __launch_bounds__(kBlock, 6) k_select_small(SampleLayer p) {
    __shared__ RunLds runs[kWavesPerBlock];
    const int wid = uniform_i32(threadIdx.x / kWave);
    RunLds& L = runs[wid];
    const int lane = lane_id();
    const int64_t fcount = p.ctl->fcount[p.layer];
    const int64_t out_base = p.ctl->out_base[p.layer];
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t e0 = (blockIdx.x * (int64_t)kWavesPerBlock + wid) * kWave; e0 < fcount; e0 += waves * kWave) {
        const int n = (int)(fcount - e0 < kWave ? fcount - e0 : kWave);
        uint64_t e16, e32;
        {
            EntryRun R;
            load_run<kBurn>(p, e0 + lane, lane < n, out_base, R);
            e16 = p.group16 > 0 ? ballot(lane < n && group_fits(R, p.capacity, p.group16)) : 0ull;
            e32 = p.group32 > 0 ? ballot(lane < n && group_fits(R, p.capacity, p.group32)) & ~e16 : 0ull;
            store_run(L, R, lane);
        }
        wave_lds_sync();
        uint64_t back = 0;
        if (e16) back |= select_groups<16>(p, L, e16);
        if (e32) back |= select_groups<32>(p, L, e32);
        for (; back; back &= back - 1) select_entry_small_draw(p, lds_entry(L, __ffsll((unsigned long long)back) - 1));
        wave_lds_sync();  // the next run overwrites L
    }
}

// Each wavefront takes a contiguous share of the frontier (a short run when
// the grid has more wavefronts than resident slots), loaded 64 entries at a
// time; entries of the sub-wave buckets are skipped (k_select_small).
template <bool kBurn>
__global__ void __launch_bounds__(kBlock) k_select(SampleLayer p) {
    const int wid = uniform_i32(threadIdx.x / kWave);
    const int lane = lane_id();
    const int64_t fcount = p.ctl->fcount[p.layer];
    const int64_t out_base = p.ctl->out_base[p.layer];
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t wave = blockIdx.x * (int64_t)kWavesPerBlock + wid;
    const int64_t per = (fcount + waves - 1) / waves;
    const int64_t lo = wave * per < fcount ? wave * per : fcount;
    const int64_t hi = lo + per < fcount ? lo + per : fcount;
    const int32_t bound = p.group32 > p.group16 ? p.group32 : p.group16;
    for (int64_t e0 = lo; e0 < hi; e0 += kWave) {
        const int n = (int)(hi - e0 < kWave ? hi - e0 : kWave);
        EntryRun R;
        load_run<kBurn>(p, e0 + lane, lane < n, out_base, R);
        uint64_t todo = ballot(lane < n && R.c != 0 && !(bound > 0 && group_fits(R, p.capacity, bound)));
        for (; todo; todo &= todo - 1) select_entry(p, run_entry(R, __ffsll((unsigned long long)todo) - 1));
    }
}

// ------------------------------------------------------ long-list path
// Chunk prefix table, once per graph and weight array: one wavefront per
// list longer than kWaveMaxD, chunk by chunk (coalesced loads, LDS
// transpose, one 16-weight group per lane, a 64-lane scan): row
// (b >> kTabShift) + j holds the inclusive group prefixes of chunk j of the
// list starting at edge b. A list of d > 512 weights spans at least
// floor(d / 512) >= ceil(d / 1024) rows of 512 edges, so the rows of
// different lists never meet, and every row is below (m >> kTabShift).
// ctab (may be null) gets the list's running total at the end of each chunk:
// ctab[(b >> kTabShift) + j] = total weight of chunks 0..j.
__global__ void __launch_bounds__(kBlock) k_chunk_table(RowPtr rowptr,
                                                        const uint32_t* __restrict__ w, int64_t n,
                                                        uint64_t* __restrict__ tab, uint64_t* __restrict__ ctab) {
    __shared__ uint32_t tiles[kWavesPerBlock][kTilePad];
    const int wid = uniform_i32(threadIdx.x / kWave);
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t v = blockIdx.x * (int64_t)kWavesPerBlock + wid; v < n; v += waves) {
        const int64_t b = uniform_i64(rowptr[v]);
        const int64_t d = uniform_i64(rowptr[v + 1]) - b;
        if (d <= kWaveMaxD) continue;
        uint64_t* row = tab + (b >> kTabShift) * kChunkGroups;
        uint64_t run = 0;
        for (int64_t j = 0; j < chunks_of(d); ++j) {
            const int64_t len = d - j * kChunk < kChunk ? d - j * kChunk : kChunk;
            const uint64_t s = tile_group_sums(w + b + j * kChunk, 0, len, tiles[wid]);
            const uint64_t incl = wave_incl_scan_u64(s);
            row[j * kChunkGroups + lane] = incl;
            run += readlane_u64(incl, kWave - 1);
            if (ctab && lane == 0) ctab[(b >> kTabShift) + j] = run;
        }
    }
}

// The group of chunk row `row` (64 inclusive group prefixes) that holds r,
// given the total acc before the chunk: the first i with acc + row[i] > r,
// and the prefix before it. Two rounds of eight independent loads (octant
// ends, then the octant) instead of a six-step binary search.
__device__ __forceinline__ int32_t row_group(const uint64_t* __restrict__ row, uint64_t acc, uint64_t r,
                                             uint64_t& before) {
    uint64_t ends[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ends[q] = row[8 * q + 7];
    int32_t o = 0;
#pragma unroll
    for (int q = 0; q < 7; ++q) o += acc + ends[q] <= r ? 1 : 0;  // r lies inside the chunk: octant 7 ends past it
    uint64_t g8[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) g8[k] = row[8 * o + k];
    int32_t c = 0;
    before = 0;
    for (int q = 0; q < 8; ++q)
        if (q < o) before = ends[q];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const bool le = acc + g8[k] <= r;
        c += le ? 1 : 0;
        before = le ? g8[k] : before;
    }
    return 8 * o + c;
}

// Per-lane search of a long list through its chunk prefixes (pass 1) and a
// coarse LDS table over units of 2^shift chunks: tab[u] = total weight of
// the chunks before unit u, tab[nu] = W. Finds the unit by binary search in
// LDS, the chunk by a walk over the unit's chunk totals, the group by binary
// search in the chunk's G row and the candidate by scanning the group's
// weights (global memory / L2).
// A list's walk guide (when the graph has one for its weight array): its
// buckets and edge records, total W and bucket shift.
struct GuidePool {
    const WalkBucket* G;
    const WalkEdge* er;
    uint64_t W, K;
    int64_t d;
    int sh;
};

// m = max{i : S_i <= r} with S_m and b_m through the walk guide, per lane:
// the bracket [G[k].pos, G[k+1].pos] of bucket k = r >> s (every position
// before it ends at or below k * 2^s <= r; its last ends past (k+1) * 2^s,
// or is the list's last), then the bracket's edge records 8 at a time
// (positions past its end read the end, whose prefix exceeds r):
// m = lo + #{j : S_(lo+j+1) <= r}, S_m = S_(m+1) - b_m. Two dependent loads
// for a bracket of up to 8 positions, whatever the list's length.
__device__ __forceinline__ void guide_search(const GuidePool& gp, uint64_t r, int64_t& m, uint64_t& Sm,
                                             uint32_t& bm) {
    const uint64_t k = r >> gp.sh;
    const bool last = k + 1 >= gp.K;
    int64_t lo = gp.G[k].pos;
    const uint32_t p1 = gp.G[last ? k : k + 1].pos;
    const int64_t hi = last ? gp.d - 1 : (int64_t)p1;
    for (;;) {
        uint64_t S[8];
        uint32_t b[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t q = lo + j < hi ? lo + j : hi;
            S[j] = gp.er[q].S;
            b[j] = gp.er[q].w;
        }
        int c = 0;
#pragma unroll
        for (int j = 0; j < 7; ++j) c += S[j] <= r ? 1 : 0;
        if (c < 7 || lo + 7 >= hi) {
            uint64_t s = S[0];
            uint32_t x = b[0];
#pragma unroll
            for (int j = 1; j < 8; ++j) {
                s = c == j ? S[j] : s;
                x = c == j ? b[j] : x;
            }
            m = lo + c;
            Sm = s - x;
            bm = x;
            return;
        }
        lo += 7;
    }
}

struct UnitPool {
    const uint64_t* tab;    // LDS, nu + 1 entries
    int64_t nu;
    int shift;
    int64_t nch;            // chunks of the list
    const uint64_t* G;      // G rows of the list's chunks
    const uint32_t* w;      // weights of the list
    int64_t d;
};

__device__ __forceinline__ void unit_search(const UnitPool& pl, uint64_t r, int64_t& m, uint64_t& Sm,
                                            uint32_t& bm) {
    int64_t lo = 0, hi = pl.nu;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (pl.tab[mid] <= r) lo = mid;
        else hi = mid;
    }
    uint64_t acc = pl.tab[lo];
    int64_t j = lo << pl.shift;
    const int64_t jend = ((lo + 1) << pl.shift) < pl.nch ? ((lo + 1) << pl.shift) : pl.nch;
    for (; j + 1 < jend; ++j) {  // chunk totals of the unit
        const uint64_t t = pl.G[j * kChunkGroups + kChunkGroups - 1];
        if (acc + t > r) break;
        acc += t;
    }
    uint64_t before;
    const int32_t ghi = row_group(pl.G + j * kChunkGroups, acc, r, before);
    const int64_t i = j * kChunk + (int64_t)ghi * 16;
    const int64_t end = i + 16 < pl.d ? i + 16 : pl.d;
    fine_scan_global(pl.w, i, end, acc + before, r, m, Sm, bm);
}

// One wavefront per long list. Lists of up to kGroupTabD weights get a
// group-level table (C[t] = weight before group t, from the chunk totals and
// the G rows), searched like the wavefront path with the group's weights
// read from global memory; longer lists get a unit-level table (UnitPool).
// The G rows come from the graph's chunk prefix table, or for a list of at
// most kWaveMaxD weights (wide total) from its one chunk reduced here.
constexpr int kBigTab = 512;
constexpr int64_t kGroupTabD = (int64_t)kBigTab * 16;

__device__ void select_big_entry(const SampleLayer& p, const EntryInfo& E, uint64_t* tab) {
    const int lane = lane_id();
    if (E.c == 0) return;
    if (E.o + E.c > p.capacity) {
        if (lane == 0) p.ctl->overflow = 1;
        return;
    }
    const int64_t d = E.d;
    const Key key{(uint32_t)E.key, (uint32_t)(E.key >> 32)};
    const uint32_t c0 = E.c0, c1 = (uint32_t)p.layer, c2 = (uint32_t)E.v;
    const bool ew = E.kind == kEdgeWeight;
    const WalkBucket* gb = ew ? p.g.wgd_ew : p.g.wgd_deg;
    const WalkEdge* ge = ew ? p.g.wrec_ew : p.g.wrec_deg;
    if (gb && ge) {  // the list's walk guide: no table to build, two loads a draw
        const uint64_t W = ld_uniform((ew ? p.g.wtot_ew : p.g.wtot_deg) + E.v);
        const int sh = guide_shift(W, d);
        const GuidePool gp{gb + guide_base(E.beg, E.v), ge + E.beg, W, ((W - 1) >> sh) + 1, d, sh};
        const auto search = [&gp](uint64_t r, int64_t& m, uint64_t& Sm, uint32_t& bm) {
            guide_search(gp, r, m, Sm, bm);
        };
        emit_slots(p, E, draw_slots(key, c0, c1, c2, E.k, p.rounds, W, search, search));
        return;
    }
    const int64_t nch = chunks_of(d);
    const uint32_t* w = (E.kind == kEdgeWeight ? p.g.ew : p.g.degw) + E.beg;
    const uint64_t* G = (E.kind == kEdgeWeight ? p.g.gtab_ew : p.g.gtab_deg) + (E.beg >> kTabShift) * kChunkGroups;
    const bool onchip = d <= kWaveMaxD;  // one chunk, not in the table
    int64_t pos;
    if (d <= kGroupTabD) {
        const int64_t nc = (d + 15) / 16;
        uint64_t rows[kGroupTabD / kChunk];
        uint64_t tj;
        if (onchip) {  // (rare) group sums straight from the list, lane = group
            const int64_t i0 = (int64_t)lane * 16;
            uint64_t s = 0;
#pragma unroll 4
            for (int q = 0; q < 16; ++q) s += i0 + q < d ? w[i0 + q] : 0u;
            rows[0] = wave_incl_scan_u64(s);
#pragma unroll
            for (int j = 1; j < kGroupTabD / kChunk; ++j) rows[j] = 0ull;
            tj = lane == 0 ? readlane_u64(rows[0], kWave - 1) : 0ull;
        } else {
#pragma unroll
            for (int j = 0; j < kGroupTabD / kChunk; ++j) rows[j] = j < nch ? G[j * kChunkGroups + lane] : 0ull;
            tj = lane < nch ? G[lane * kChunkGroups + kChunkGroups - 1] : 0ull;
        }
        const uint64_t cincl = wave_incl_scan_u64(tj);
        const uint64_t cex = cincl - tj;
#pragma unroll
        for (int j = 0; j < kGroupTabD / kChunk; ++j) {
            const uint64_t base = readlane_u64(cex, j);
            const int64_t t = (int64_t)j * kChunkGroups + lane;
            if (j < nch && t < nc) tab[t + 1] = base + rows[j];
        }
        if (lane == 0) tab[0] = 0;
        const uint64_t W = readlane_u64(cincl, (int)nch - 1);
        wave_lds_sync();
        const CoarsePool pl{tab, nc, 16, d, w};
        const auto search = [&pl](uint64_t r, int64_t& m, uint64_t& Sm, uint32_t& bm) {
            coarse_search(pl, r, m, Sm, bm);
        };
        pos = draw_slots(key, c0, c1, c2, E.k, p.rounds, W, search, search);
    } else {
        int shift = 0;
        while (((nch + (1ll << shift) - 1) >> shift) > kBigTab) ++shift;
        const int64_t nu = (nch + (1ll << shift) - 1) >> shift;
        uint64_t carry = 0;
        for (int64_t u0 = 0; u0 < nu; u0 += kWave) {
            const int64_t u = u0 + lane;
            uint64_t s = 0;
            if (u < nu) {
                const int64_t j0 = u << shift;
                const int64_t j1 = j0 + (1ll << shift) < nch ? j0 + (1ll << shift) : nch;
                for (int64_t j = j0; j < j1; ++j) s += G[j * kChunkGroups + kChunkGroups - 1];
            }
            const uint64_t incl = wave_incl_scan_u64(s);
            if (u < nu) tab[u + 1] = carry + incl;
            carry += readlane_u64(incl, kWave - 1);
        }
        if (lane == 0) tab[0] = 0;
        wave_lds_sync();
        const UnitPool pl{tab, nu, shift, nch, G, w, d};
        const auto search = [&pl](uint64_t r, int64_t& m, uint64_t& Sm, uint32_t& bm) {
            unit_search(pl, r, m, Sm, bm);
        };
        pos = draw_slots(key, c0, c1, c2, E.k, p.rounds, carry, search, search);
    }
    emit_slots(p, E, pos);
    wave_lds_sync();  // the table is rewritten by the wave's next list
}

template <bool kBurn>
__global__ void __launch_bounds__(kBlock) k_select_big(SampleLayer p) {
    __shared__ uint64_t tabs[kWavesPerBlock][kBigTab + 1];
    const int wid = uniform_i32(threadIdx.x / kWave);
    const int lane = lane_id();
    const int64_t nb = (int64_t)p.ctl->nbig[p.layer];
    const int64_t out_base = p.ctl->out_base[p.layer];
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t wave = blockIdx.x * (int64_t)kWavesPerBlock + wid;
    const int64_t per = (nb + waves - 1) / waves;
    const int64_t lo = wave * per < nb ? wave * per : nb;
    const int64_t hi = lo + per < nb ? lo + per : nb;
    for (int64_t h0 = lo; h0 < hi; h0 += kWave) {
        const int n = (int)(hi - h0 < kWave ? hi - h0 : kWave);
        const bool valid = lane < n;
        const int64_t pos = valid ? p.bigs[h0 + lane] : 0;
        EntryRun R;
        load_run<kBurn>(p, pos, valid, out_base, R);
        for (int j = 0; j < n; ++j) select_big_entry(p, run_entry(R, j), tabs[wid]);
    }
}

// ------------------------------------------------------ layer sampling
// One wavefront per instance, every layer in the kernel (Section II-A:
// layer sampling selects a constant number of neighbors for the whole
// frontier). Per layer: per frontier vertex its list's total bias and
// length, two exclusive prefixes over the frontier in LDS (bias and
// position), then k slots drawn like one list (rounds in slot order, direct
// draws) with counter (instance id, layer, 0xFFFFFFFF, slot | round << 16):
// a draw r finds its frontier vertex by binary search in the bias prefix and
// its neighbor in that list (list_search; the position itself if unbiased). Picks not visited, deduplicated and sorted, form the next
// frontier (at most 64 vertices).
__device__ __forceinline__ int32_t lds_upper(const uint64_t* a, int32_t n, uint64_t r) {
    // largest f in [0, n) with a[f] <= r (a[0] = 0 <= r)
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (a[mid] <= r) lo = mid;
        else hi = mid;
    }
    return lo;
}

// m = max{i : S_i <= r} inside one weighted list (weights w, first edge beg,
// length d, prefix acc before it), with S_m and b_m: a scan of the list for
// up to kWaveMaxD weights, else through the graph's chunk prefix table
// (chunk totals, then the chunk's group prefixes, then one group).
__device__ __forceinline__ void list_search(const uint32_t* __restrict__ w, const uint64_t* __restrict__ gtab,
                                            int64_t beg, int64_t d, uint64_t acc, uint64_t r, int64_t& m,
                                            uint64_t& Sm, uint32_t& bm) {
    if (d <= kWaveMaxD) {
        fine_scan_global(w, 0, d, acc, r, m, Sm, bm);
        return;
    }
    const uint64_t* G = gtab + (beg >> kTabShift) * kChunkGroups;
    const int64_t nch = chunks_of(d);
    int64_t j = 0;
    for (; j + 1 < nch; ++j) {
        const uint64_t t = G[j * kChunkGroups + kChunkGroups - 1];
        if (acc + t > r) break;
        acc += t;
    }
    uint64_t before;
    const int32_t ghi = row_group(G + j * kChunkGroups, acc, r, before);
    const int64_t i = j * kChunk + (int64_t)ghi * 16;
    fine_scan_global(w, i, i + 16 < d ? i + 16 : d, acc + before, r, m, Sm, bm);
}

// LDS of one wavefront, sized by the call's largest seed set mf and its
// layers. A frontier holds the seeds, then at most 64 picks: cf = max(mf, 64)
// entries. The two prefixes (uint64, cf + 1 each), then the frontier (cf),
// the visited list (mf + 64 per layer) and the picks (64).
__host__ __device__ inline int32_t layer_frontier_cap(int32_t mf) { return mf > kWave ? mf : kWave; }
inline size_t layer_lds_bytes(int32_t mf, int32_t L) {
    const size_t cf = (size_t)layer_frontier_cap(mf);
    return 2 * sizeof(uint64_t) * (cf + 1) + sizeof(int32_t) * (cf + (size_t)mf + 64 * (size_t)L + kWave);
}

__global__ void __launch_bounds__(kWave) k_layer_sample(LayerParams p) {
    extern __shared__ __align__(16) unsigned char layer_lds[];
    const int32_t cf = layer_frontier_cap(p.max_f);
    uint64_t* Wp = (uint64_t*)layer_lds;
    uint64_t* Dp = Wp + (cf + 1);
    int32_t* F = (int32_t*)(Dp + (cf + 1));
    int32_t* vis = F + cf;
    int32_t* pk = vis + p.max_f + 64 * p.L;  // this layer's picks by slot
    const int lane = lane_id();
    const Key key{p.k0, p.k1};
    const uint32_t* wts = p.bias == kEdgeWeight ? p.g.ew : p.g.degw;
    const int32_t* ppos = p.bias == kEdgeWeight ? p.g.ppos_ew : p.g.ppos_deg;
    const uint64_t* wtot = p.bias == kEdgeWeight ? p.g.wtot_ew : p.g.wtot_deg;
    const uint64_t* gtab = p.bias == kEdgeWeight ? p.g.gtab_ew : p.g.gtab_deg;
    for (int64_t i = blockIdx.x; i < p.num_instances; i += gridDim.x) {
        const int64_t o0 = uniform_i64(p.seed_off[i]);
        int32_t nf = (int32_t)(uniform_i64(p.seed_off[i + 1]) - o0);  // <= kMaxPool (checked by the host)
        const uint32_t iid = (uint32_t)(p.instance_base + (uint64_t)i);
        bool bad = false;
        for (int32_t f = lane; f < nf; f += kWave) {
            const int32_t v = p.seeds[o0 + f];
            const int32_t prev = f > 0 ? p.seeds[o0 + f - 1] : -1;
            bad |= v < 0 || (int64_t)v >= p.g.n || v <= prev;
            F[f] = v;
            vis[f] = v;
        }
        if (ballot(bad)) {  // outputs of the call are unspecified; the host reports the error
            if (lane == 0) *p.bad = 1;
            wave_lds_sync();
            continue;
        }
        int32_t nvis = nf;
        wave_lds_sync();
        for (int32_t l = 0; l < p.L; ++l) {
            const int32_t k = p.fan[l];
            int32_t* src = p.src + (i * p.L + l) * p.K;
            int32_t* dst = p.dst + (i * p.L + l) * p.K;
            // totals per frontier vertex, then both prefixes, 64 vertices at a time
            uint64_t carry_w = 0, carry_d = 0, npos = 0;
            if (lane == 0) Wp[0] = Dp[0] = 0;
            for (int32_t f0 = 0; f0 < nf; f0 += kWave) {
                const int32_t f = f0 + lane;
                uint64_t wv = 0, dv = 0, pv = 0;
                if (f < nf) {
                    const int32_t v = F[f];
                    const int64_t beg = p.g.rowptr[v];
                    dv = (uint64_t)(p.g.rowptr[v + 1] - beg);
                    if (p.bias == kUniform) {
                        wv = pv = dv;
                    } else {
                        wv = wtot[v];
                        pv = (uint64_t)(ppos[v] & ~kWideList);
                    }
                }
                const uint64_t iw = wave_incl_scan_u64(wv), id = wave_incl_scan_u64(dv);
                if (f < nf) {
                    Wp[f + 1] = carry_w + iw;
                    Dp[f + 1] = carry_d + id;
                }
                carry_w += readlane_u64(iw, kWave - 1);
                carry_d += readlane_u64(id, kWave - 1);
                npos += wave_sum_u64(pv);
            }
            wave_lds_sync();
            const uint64_t W = carry_w;
            const int32_t c = W == 0 ? 0 : ((uint64_t)k >= npos ? (int32_t)npos : k);
            int64_t pos = -1;  // this lane's pool position (slot lane < c)
            if (c > 0 && (uint64_t)k >= npos) {
                // every positive position, pool order
                int32_t run = 0;
                for (int32_t f = 0; f < nf; ++f) {
                    const int64_t beg = p.g.rowptr[F[f]];
                    const int64_t d = (int64_t)(Dp[f + 1] - Dp[f]);
                    for (int64_t b0 = 0; b0 < d; b0 += kWave) {
                        const int64_t e = b0 + lane;
                        const bool posv = e < d && (p.bias == kUniform || wts[beg + e] > 0);
                        const uint64_t m = ballot(posv);
                        const int32_t slot = run + __popcll(m & lanemask_lt());
                        if (posv) {
                            const int32_t nb = p.g.col[beg + e];
                            src[slot] = F[f];
                            dst[slot] = nb;
                            pk[slot] = nb;
                        }
                        run += __popcll(m);
                    }
                }
            } else if (c > 0) {
                const auto search = [&](uint64_t r, int64_t& m, uint64_t& Sm, uint32_t& bm) {
                    const int32_t f = lds_upper(Wp, nf, r);
                    if (p.bias == kUniform) {
                        m = (int64_t)r;
                        Sm = r;
                        bm = 1;
                    } else {
                        const int32_t v = F[f];
                        const int64_t beg = p.g.rowptr[v];
                        int64_t ml = 0;
                        list_search(wts + beg, gtab, beg, (int64_t)(Dp[f + 1] - Dp[f]), Wp[f], r, ml, Sm, bm);
                        m = (int64_t)Dp[f] + ml;
                    }
                };
                pos = draw_slots(key, iid, (uint32_t)l, 0xFFFFFFFFu, c, p.rounds, W, search, search);
                if (lane < c) {
                    const int32_t f = lds_upper(Dp, nf, (uint64_t)pos);
                    const int32_t v = F[f];
                    const int32_t nb = p.g.col[p.g.rowptr[v] + (pos - (int64_t)Dp[f])];
                    src[lane] = v;
                    dst[lane] = nb;
                    pk[lane] = nb;
                }
            }
            for (int32_t j = c + lane; j < p.K; j += kWave) src[j] = dst[j] = -1;
            if (lane == 0) p.counts[i * p.L + l] = c;
            // next frontier: the picks, deduplicated, minus visited, sorted
            wave_lds_sync();
            const int32_t x = lane < c ? pk[lane] : -1;
            bool keep = lane < c;
            for (int32_t q = 0; q < nvis && keep; ++q) keep = vis[q] != x;
            for (int j = 0; j < kWave; ++j) {
                const int32_t y = readlane_i32(x, j);
                if (j < lane && y == x) keep = false;
            }
            const uint64_t km = ballot(keep);
            int32_t rank = 0;
            for (int j = 0; j < kWave; ++j) {
                const int32_t y = readlane_i32(x, j);
                if (((km >> j) & 1ull) && y < x) ++rank;
            }
            wave_lds_sync();
            if (keep) {
                F[rank] = x;
                vis[nvis + rank] = x;
            }
            nf = __popcll(km);
            nvis += nf;
            wave_lds_sync();
        }
    }
}

__global__ void k_call_setup(uint32_t* __restrict__ ctl, int64_t nctl, const uint32_t* __restrict__ host_tab,
                             uint32_t* __restrict__ tab, int64_t ntab) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nctl; i += stride) ctl[i] = 0u;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntab; i += stride) tab[i] = host_tab[i];
}

// End of a call: clear the visited bits of every frontier entry, and hand
// the control block to the host.
__global__ void k_clear_visited(ClearVisited c) {
    if (blockIdx.x == 0) {
        constexpr int kWords = (int)(sizeof(SampleCtl) / 4);
        const uint32_t* from = (const uint32_t*)c.ctl;
        uint32_t* to = (uint32_t*)c.host_ctl;
        for (int i = threadIdx.x; i < kWords; i += blockDim.x) to[i] = from[i];
        __threadfence_system();
    }
    for (int l = 0; l < c.num_layers; ++l) {
        const int64_t fcount = c.fcount[l];
        const int32_t* __restrict__ fv = c.fv[l];
        const int32_t* __restrict__ fi = c.fi[l];
        for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < fcount;
             e += (int64_t)gridDim.x * blockDim.x)
            c.visited[(int64_t)fi[e] * c.nwp + (fv[e] >> 5)] = 0u;
    }
}

// Frontier entries and their edges per vertex-range partition of a layer
// (out-of-memory schedule): partition p holds vertices [bounds[p],
// bounds[p+1]); block-local sums in LDS, one atomic per partition and block.
constexpr int kMaxPartitions = 64;

__global__ void __launch_bounds__(kBlock) k_partition_work(const int32_t* __restrict__ fv,
                                                           const int32_t* __restrict__ cnt, const SampleCtl* ctl,
                                                           int32_t layer, const int64_t* __restrict__ bounds,
                                                           int32_t np, unsigned long long* __restrict__ work) {
    __shared__ unsigned long long s_work[2 * kMaxPartitions];
    for (int i = threadIdx.x; i < 2 * kMaxPartitions; i += blockDim.x) s_work[i] = 0ull;
    __syncthreads();
    const int64_t fcount = ctl->fcount[layer];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < fcount;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = fv[e];
        int32_t lo = 0, hi = np;  // the partition: largest p with bounds[p] <= v
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (bounds[mid] <= v) lo = mid;
            else hi = mid;
        }
        atomicAdd(&s_work[2 * lo], 1ull);
        atomicAdd(&s_work[2 * lo + 1], (unsigned long long)cnt[e]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * np; i += blockDim.x)
        if (s_work[i]) atomicAdd(&work[i], s_work[i]);
}

}  // namespace

// ---------------------------------------------------------------- launchers}  // namespace

// ---------------------------------------------------------------- launchers
void launch_partition_work(const int32_t* fv, const int32_t* cnt, const SampleCtl* ctl, int32_t layer,
                           int64_t capacity, const int64_t* bounds, int32_t np, unsigned long long* work,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_partition_work, dim3(grid_for(capacity, kBlock, 1024)), dim3(kBlock), 0, s, fv, cnt, ctl,
                       layer, bounds, np, work);
}

void launch_scatter_segments(const int32_t* src, const int32_t* dst, const int64_t* off, int64_t nseg,
                             int64_t total, int32_t* const* to_src, int32_t* const* to_dst, hipStream_t s) {
    if (nseg <= 0 || total <= 0) return;
    hipLaunchKernelGGL(k_scatter_segments, dim3(grid_for(total, kBlock, 8192)), dim3(kBlock), 0, s, src, dst, off,
                       nseg, to_src, to_dst);
}

void launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, kBlock, 65536)), dim3(kBlock), 0, s, p, value, count);
}

void launch_degree_weights(RowPtr rowptr, const int32_t* col, int64_t m, uint32_t* degw,
                           hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_degree_weights, dim3(grid_for(m, kBlock, 65536)), dim3(kBlock), 0, s, rowptr, col,
                       m, degw);
}

void launch_positive_counts(RowPtr rowptr, const uint32_t* w, int64_t n, int32_t* ppos, uint64_t* wtot,
                            hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_positive_counts, dim3(grid_for(n, kWavesPerBlock, 65536)), dim3(kBlock), 0, s,
                       rowptr, w, n, ppos, wtot);
}

void launch_mark_seeds(const int32_t* seeds, int64_t num_seeds, const int64_t* seed_offsets, int32_t ni,
                       int64_t n, uint32_t* next, int64_t nwp, uint32_t* summ, int64_t nsw, SampleCtl* ctl,
                       hipStream_t s) {
    if (num_seeds <= 0) return;
    hipLaunchKernelGGL(k_mark_seeds, dim3(grid_for(num_seeds, kBlock, 65536)), dim3(kBlock), 0, s, seeds,
                       num_seeds, seed_offsets, ni, n, next, nwp, summ, nsw, ctl);
}

// Bitmap words per thread of the frontier build: one up to 2^20 words (one
// instance of a 2^25-vertex graph), 16 above.
static int frontier_build_words(int64_t words) { return words > (int64_t(1) << 20) ? 16 : 1; }

int64_t frontier_build_blocks(int64_t words) {
    const int64_t per = (int64_t)kBlock * frontier_build_words(words);
    const int64_t nb = (words + per - 1) / per;
    return nb > 0 ? nb : 1;
}

void launch_frontier_build(const FrontierBuild& fb, hipStream_t s, LaunchEvents ev) {
    if (fb.summ) {  // sparse: compact the summary, then one thread per dirty word
        hipLaunchKernelGGL(k_dirty_compact, dim3((unsigned)fb.nb_dirty), dim3(kBlock), 0, s, fb);
        launch_kernel(fb.burn ? k_frontier_build<1, 1, true, true> : k_frontier_build<1, 1, false, true>,
                      dim3((unsigned)fb.nb), dim3(kBlock), s, ev, fb);
        return;
    }
    const bool wide = frontier_build_words(fb.nwords) == 16;
    if (fb.burn)
        launch_kernel(wide ? k_frontier_build<4, 4, true, false> : k_frontier_build<1, 1, true, false>,
                      dim3((unsigned)fb.nb), dim3(kBlock), s, ev, fb);
    else
        launch_kernel(wide ? k_frontier_build<4, 4, false, false> : k_frontier_build<1, 1, false, false>,
                      dim3((unsigned)fb.nb), dim3(kBlock), s, ev, fb);
}

int64_t sparse_build_blocks(int64_t capacity) {
    const int64_t nb = (capacity + kBlock - 1) / kBlock;
    return nb > 0 ? nb : 1;
}

int64_t dirty_compact_blocks(int64_t summary_words) {
    const int64_t per = (int64_t)kBlock * 4;
    const int64_t nb = (summary_words + per - 1) / per;
    return nb > 0 ? nb : 1;
}

void launch_select(const SampleLayer& p, int grid, hipStream_t s, LaunchEvents ev) {
    launch_kernel(p.burn ? k_select<true> : k_select<false>, dim3(grid), dim3(kBlock), s, ev, p);
}

void launch_select_small(const SampleLayer& p, int grid, hipStream_t s, LaunchEvents ev) {
    launch_kernel(p.burn ? k_select_small<true> : k_select_small<false>, dim3(grid), dim3(kBlock), s, ev, p);
}

void launch_layer_sample(const LayerParams& p, hipStream_t s, LaunchEvents ev) {
    if (p.num_instances <= 0) return;
    const int grid = (int)(p.num_instances < 8192 ? p.num_instances : 8192);
    const size_t lds = layer_lds_bytes(p.max_f, p.L);
    if (ev.start || ev.stop)
        hipExtLaunchKernelGGL(k_layer_sample, dim3(grid), dim3(kWave), lds, s, ev.start, ev.stop, 0, p);
    else
        hipLaunchKernelGGL(k_layer_sample, dim3(grid), dim3(kWave), lds, s, p);
}

int64_t chunk_table_rows(int64_t m) { return (m >> kTabShift) + 1; }

void launch_chunk_table(RowPtr rowptr, const uint32_t* w, int64_t n, uint64_t* tab, uint64_t* ctab,
                        hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_chunk_table, dim3(grid_for(n, kWavesPerBlock, 65536)), dim3(kBlock), 0, s, rowptr, w, n,
                       tab, ctab);
}

void launch_select_big(const SampleLayer& p, int grid, hipStream_t s, LaunchEvents ev) {
    launch_kernel(p.burn ? k_select_big<true> : k_select_big<false>, dim3(grid), dim3(kBlock), s, ev, p);
}

void launch_clear_visited(const ClearVisited& c, hipStream_t s, LaunchEvents ev) {
    launch_kernel(k_clear_visited, dim3(grid_for(c.cap_entries, kBlock, 16384)), dim3(kBlock), s, ev, c);
}

void launch_call_setup(uint32_t* ctl, int64_t nctl, const uint32_t* host_tab, uint32_t* tab, int64_t ntab,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_call_setup, dim3(grid_for(nctl > ntab ? nctl : ntab, kBlock, 1024)), dim3(kBlock), 0, s,
                       ctl, nctl, host_tab, tab, ntab);
}

}  // namespace csaw
