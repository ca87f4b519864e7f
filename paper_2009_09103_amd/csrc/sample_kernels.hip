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
constexpr int kWin = 1024;  // LDS prefix window (uint64 entries) per wavefront

inline int grid_for(int64_t items, int per_block, int cap = 1 << 20) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ----------------------------------------------------------- block helpers
// Exclusive scan of one int64 per thread over a 256-thread block; returns the
// exclusive prefix and writes the block total to *total.
__device__ __forceinline__ int64_t block_excl_scan_i64(int64_t x, int64_t* total) {
    __shared__ int64_t wsum[kWavesPerBlock];
    const int lane = lane_id();
    const int wid = threadIdx.x / kWave;
    const uint64_t incl = wave_incl_scan_u64((uint64_t)x);
    if (lane == kWave - 1) wsum[wid] = (int64_t)incl;
    __syncthreads();
    int64_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) {
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
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t seg = (nb + 1023) / 1024;
    const int64_t b0 = t * seg, b1 = (b0 + seg < nb) ? b0 + seg : nb;
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += bs[b];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over 1024 partials
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t add = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t x = bs[b];
        bs[b] = run;
        run += x;
    }
    if (t == 1023) *total = part[1023];
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
        } else c = k;
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
// Where the wavefront finds the candidate owning r:
//   kModeUniform : S_i = i, no weights
//   kModeWindow  : full exclusive prefix S[0..d] in LDS (d <= kWin)
//   kModeCoarse  : S at every G = 64*q-th position in LDS; the owning chunk
//                  is re-read from global memory and scanned by the wave
enum { kModeUniform = 0, kModeWindow = 1, kModeCoarse = 2 };

struct Pool {
    int mode;
    int64_t d;
    int64_t beg;
    const uint32_t* w;
    const uint64_t* S;  // LDS
    int64_t nc;         // coarse chunks
    int64_t G;          // coarse chunk length
};

// Inverse transform search: m = max{i in [0,d) : S_i <= r}, with S_m and b_m.
// Per lane for the uniform and window modes (lanes with want = false are
// untouched); cooperatively, one wanted lane at a time, for the coarse mode.
__device__ __forceinline__ void its_search(const Pool& pl, bool want, uint64_t r, int64_t& m,
                                           uint64_t& Sm, uint32_t& bm) {
    if (pl.mode == kModeUniform) {
        if (want) {
            m = (int64_t)r;
            Sm = r;
            bm = 1;
        }
        return;
    }
    if (pl.mode == kModeWindow) {
        if (want) {
            int64_t lo = 0, hi = pl.d;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (pl.S[mid] <= r) lo = mid;
                else hi = mid;
            }
            m = lo;
            Sm = pl.S[lo];
            bm = (uint32_t)(pl.S[lo + 1] - pl.S[lo]);
        }
        return;
    }
    const int lane = lane_id();
    uint64_t wm = ballot(want);
    while (wm) {
        const int j = __ffsll((unsigned long long)wm) - 1;
        const uint64_t rj = readlane_u64(r, j);
        int64_t lo = 0, hi = pl.nc;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (pl.S[mid] <= rj) lo = mid;
            else hi = mid;
        }
        uint64_t acc = pl.S[lo];
        const int64_t cs = lo * pl.G;
        const int64_t ce = (cs + pl.G < pl.d) ? cs + pl.G : pl.d;
        int64_t mj = cs;
        uint64_t Smj = acc;
        uint32_t bmj = 0;
        for (int64_t base = cs; base < ce; base += kWave) {
            const int64_t idx = base + lane;
            const uint32_t x = idx < ce ? pl.w[pl.beg + idx] : 0u;
            const uint64_t incl = wave_incl_scan_u64(x);
            const uint64_t tot = readlane_u64(incl, kWave - 1);
            if (acc + tot > rj) {
                const int L = __popcll(ballot(acc + incl <= rj));
                const uint64_t inclL = readlane_u64(incl, L);
                const uint32_t xL = readlane_u32(x, L);
                mj = base + L;
                Smj = acc + inclL - xL;
                bmj = xL;
                break;
            }
            acc += tot;
        }
        if (lane == j) {
            m = mj;
            Sm = Smj;
            bm = bmj;
        }
        wm &= wm - 1;
    }
}

__device__ __forceinline__ void claim(bool do_claim, const uint32_t* visb, uint32_t* nextb, int32_t x) {
    if (!do_claim) return;
    const uint32_t bit = 1u << (x & 31);
    if (!(visb[x >> 5] & bit)) atomicOr(&nextb[x >> 5], bit);
}

__device__ void select_entry(const SampleLayer& p, int64_t e, int64_t out_base, uint64_t* S) {
    const int lane = lane_id();
    const int32_t c = uniform_i32(p.cnt[e]);
    if (c == 0) return;
    const int32_t v = uniform_i32(p.fv[e]);
    const int32_t inst = uniform_i32(p.fi[e]);
    const int64_t o = out_base + uniform_i64(p.off[e]);
    if (o + c > p.capacity) {
        if (lane == 0) p.ctl->overflow = 1;
        return;
    }
    const int32_t k = uniform_i32(p.fanout[inst]);
    const int32_t kind = uniform_i32(p.bias[inst]);
    const bool do_claim = p.fanout_next[inst] != 0;
    const int64_t beg = uniform_i64(p.g.rowptr[v]);
    const int64_t d = uniform_i64(p.g.rowptr[v + 1]) - beg;
    const uint32_t* visb = p.visited + (int64_t)inst * p.nwp;
    uint32_t* nextb = p.next + (int64_t)inst * p.nwp;
    const bool weighted = kind != kUniform;
    const uint32_t* w = kind == kEdgeWeight ? p.g.ew : p.g.degw;
    const int32_t P = weighted ? uniform_i32(kind == kEdgeWeight ? p.g.ppos_ew[v] : p.g.ppos_deg[v])
                               : (int32_t)d;
    int32_t* src = p.src + o;
    int32_t* dst = p.dst + o;

    // ---- NeighborSize >= pool: every positive-bias neighbor, list order
    if (k < 0 || k >= P) {
        if (!weighted || P == d) {
            for (int64_t j = lane; j < d; j += kWave) {
                const int32_t x = p.g.col[beg + j];
                src[j] = v;
                dst[j] = x;
                claim(do_claim, visb, nextb, x);
            }
        } else {
            int64_t run = 0;
            for (int64_t base = 0; base < d; base += kWave) {
                const int64_t idx = base + lane;
                const bool pos = idx < d && w[beg + idx] > 0;
                const uint64_t mask = ballot(pos);
                if (pos) {
                    const int64_t slot = run + __popcll(mask & lanemask_lt());
                    const int32_t x = p.g.col[beg + idx];
                    src[slot] = v;
                    dst[slot] = x;
                    claim(do_claim, visb, nextb, x);
                }
                run += __popcll(mask);
            }
        }
        return;
    }

    // ---- k < P <= d: draw k distinct candidates (k <= kMaxDrawFanout)
    Pool pl;
    pl.d = d;
    pl.beg = beg;
    pl.w = w;
    pl.S = S;
    pl.nc = 0;
    pl.G = 0;
    uint64_t W;
    wave_lds_sync();
    if (!weighted) {
        pl.mode = kModeUniform;
        W = (uint64_t)d;
    } else if (d <= kWin) {
        pl.mode = kModeWindow;
        uint64_t carry = 0;
        if (lane == 0) S[0] = 0;
        for (int64_t base = 0; base < d; base += kWave) {
            const int64_t idx = base + lane;
            const uint32_t x = idx < d ? w[beg + idx] : 0u;
            const uint64_t incl = wave_incl_scan_u64(x);
            S[idx + 1] = carry + incl;
            carry += readlane_u64(incl, kWave - 1);
        }
        W = carry;
    } else {
        pl.mode = kModeCoarse;
        int64_t q = 1;
        while ((d + kWave * q - 1) / (kWave * q) > kWin) q <<= 1;
        pl.G = kWave * q;
        pl.nc = (d + pl.G - 1) / pl.G;
        uint64_t carry = 0;
        if (lane == 0) S[0] = 0;
        for (int64_t t = 0; t < pl.nc; ++t) {
            const int64_t cs = t * pl.G;
            const int64_t ce = (cs + pl.G < d) ? cs + pl.G : d;
            uint64_t part = 0;
            for (int64_t idx = cs + lane; idx < ce; idx += kWave) part += w[beg + idx];
            carry += wave_sum_u64(part);
            if (lane == 0) S[t + 1] = carry;
        }
        W = carry;
    }
    wave_lds_sync();

    const Key key{p.k0, p.k1};
    const uint32_t c0 = (uint32_t)(p.instance_base + (uint64_t)inst);
    const uint32_t c1 = (uint32_t)p.layer;
    const uint32_t c2 = (uint32_t)v;
    const bool active = lane < k;
    bool held = false;
    int64_t pos = 0;
    uint64_t Spos = 0;
    uint32_t bpos = 0;

    // repeated sampling rounds; lowest slot wins a collision
    for (int a = 0; a < kRounds; ++a) {
        const bool open = active && !held;
        if (ballot(open) == 0) break;
        uint64_t r = 0;
        if (open) r = draw(key, c0, c1, c2, (uint32_t)lane | ((uint32_t)a << 16), W);
        int64_t m = -1;
        uint64_t Sm = 0;
        uint32_t bm = 0;
        its_search(pl, open, r, m, Sm, bm);
        const uint64_t heldmask = ballot(held);
        const int64_t val = held ? pos : m;
        bool reject = false;
        for (int q = 0; q < k; ++q) {
            const int64_t pq = readlane_i64(val, q);
            const bool qheld = (heldmask >> q) & 1ull;
            if (q != lane && pq == m && (qheld || q < lane)) reject = true;
        }
        if (open && !reject) {
            held = true;
            pos = m;
            Spos = Sm;
            bpos = bm;
        }
    }

    // direct draws from the prefix without the held candidates, slot order
    uint64_t heldmask = ballot(held);
    const uint64_t activemask = ballot(active);
    uint64_t openmask = activemask & ~heldmask;
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
            const uint64_t skip = wave_sum_u64((held && Spos - before <= r0) ? (uint64_t)bpos : 0ull);
            const uint64_t r = r0 + skip;
            int64_t m = 0;
            uint64_t Sm = 0;
            uint32_t bm = 0;
            its_search(pl, pl.mode == kModeCoarse ? lane == j : true, r, m, Sm, bm);
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

    if (active) {
        const int32_t x = p.g.col[beg + pos];
        src[lane] = v;
        dst[lane] = x;
        claim(do_claim, visb, nextb, x);
    }
}

__global__ void __launch_bounds__(kBlock) k_select(SampleLayer p) {
    __shared__ uint64_t lds[kWavesPerBlock][kWin + 1];
    const int wid = threadIdx.x / kWave;
    uint64_t* S = lds[wid];
    const int64_t fcount = p.ctl->fcount[p.layer];
    const int64_t out_base = p.ctl->out_base[p.layer];
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t e = blockIdx.x * (int64_t)kWavesPerBlock + wid; e < fcount; e += waves)
        select_entry(p, e, out_base, S);
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
        (void)hipMemsetAsync(fcount_out, 0, sizeof(int64_t), s);
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
        (void)hipMemsetAsync(total_out, 0, sizeof(int64_t), s);
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
