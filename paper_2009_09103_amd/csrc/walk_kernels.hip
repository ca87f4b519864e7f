// walk_kernels.hip -- gfx950 kernels of random walks (DeepWalk, biased
// DeepWalk, node2vec; Section II-A of the paper).
//
// A walk is a chain of one-draw selections (NeighborSize 1, with
// replacement). The step loop runs inside the kernel: walkers are
// independent, so no host round trip is needed between steps.
//   - unbiased walks: one lane per walker (a step is two row-offset loads,
//     one Philox draw and one neighbor load);
//   - edge-weight and degree-biased walks through the graph's walk guide
//     (exact per-edge prefixes and a bucket table per list; a step is three
//     rounds of loads): one lane per walker in launches of at least
//     kLaneWalkMin walkers, else one wavefront per walker (lists of at most
//     512 scanned whole); with the guide off, one wavefront per walker
//     through the chunk tables;
//   - other biased walks: one wavefront per walker; pass 1 streams the
//     biases of N(v) into a coarse prefix table in LDS, r is drawn in [0, W),
//     and pass 2 rescans only the group of the table that holds r.
//   - node2vec: the bias of x in N(v) needs "is x adjacent to the previous
//     vertex t"; adjacency lists are sorted, so N(v) is merged with N(t)
//     (or, for a much longer N(t), each candidate binary-searches it).
#include "device_common.h"
#include "kernels.h"

namespace csaw {

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// Restart / jump rule of a step: draws x in [0, 2^32) with counter (walker,
// step, v, 2); below restart the walker returns to its start, below
// restart + jump it moves to a vertex drawn in [0, n) with counter (walker,
// step, v, 3). Returns whether the step is such a move.
__device__ __forceinline__ bool walk_move(const WalkParams& p, Key key, uint32_t c0, int32_t s, int32_t v,
                                         int32_t start, int32_t& to) {
    if ((p.restart | p.jump) == 0) return false;
    const uint64_t x = draw(key, c0, (uint32_t)s, (uint32_t)v, 2u, 1ull << 32);
    if (x < (uint64_t)p.restart) {
        to = start;
        return true;
    }
    if (x < (uint64_t)p.restart + p.jump) {
        to = (int32_t)draw(key, c0, (uint32_t)s, (uint32_t)v, 3u, (uint64_t)p.g.n);
        return true;
    }
    return false;
}

// Walker w's Philox key, length, walker id (counter word 0), path row and
// step counter: from the call, or from its request's entries in a batch.
struct WalkerCtx {
    Key key;
    int32_t length;
    uint32_t c0;
    int32_t* path;
    unsigned long long* steps;
};

__device__ __forceinline__ WalkerCtx walker_ctx(const WalkParams& p, int64_t w) {
    WalkerCtx c;
    if (p.batch.req) {
        const int32_t q = p.batch.req[w];
        const uint64_t k = p.batch.key[q];
        c.key = Key{(uint32_t)k, (uint32_t)(k >> 32)};
        c.length = p.batch.length[q];
        const int64_t i = w - p.batch.first[q];
        c.c0 = (uint32_t)(p.batch.base[q] + (uint64_t)i);
        c.path = p.paths + p.batch.path[q] + i * ((int64_t)c.length + 1);
        c.steps = p.batch.steps + q;
    } else {
        c.key = Key{p.k0, p.k1};
        c.length = p.length;
        c.c0 = (uint32_t)(p.walker_ids ? p.walker_ids[w] : p.walker_base + (uint64_t)w);
        c.path = p.paths + w * ((int64_t)p.length + 1);
        c.steps = p.steps;
    }
    return c;
}

// kMH: Metropolis-Hastings (Section II-A): the uniform pick u is a proposal,
// accepted iff x * deg(u) < deg(v) * 2^32 for x in [0, 2^32) drawn with
// counter (walker id, step, v, 4); a rejected proposal is a step that stays.
template <bool kMH>
__global__ void __launch_bounds__(kBlock) k_walk_uniform(WalkParams p) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w0 = blockIdx.x * (int64_t)blockDim.x; w0 < p.num_walkers; w0 += stride) {
        const int64_t w = w0 + threadIdx.x;
        int64_t my_steps = 0;
        unsigned long long* my_counter = p.steps;
        if (w < p.num_walkers) {
            const WalkerCtx wc = walker_ctx(p, w);
            const Key key = wc.key;
            const int64_t L1 = (int64_t)wc.length + 1;
            int32_t* path = wc.path;
            my_counter = wc.steps;
            int32_t v = p.starts[w];
            int32_t s = 0;
            if (v < 0 || (int64_t)v >= p.g.n) {
                *p.bad_start = 1;
                for (int64_t q = 0; q < L1; ++q) path[q] = -1;
            } else {
                path[0] = v;
                const int32_t start = v;
                const uint32_t c0 = wc.c0;
                for (; s < wc.length; ++s) {
                    int32_t to;
                    if (walk_move(p, key, c0, s, v, start, to)) {
                        v = to;
                        path[s + 1] = v;
                        continue;
                    }
                    const int64_t beg = p.g.rowptr[v];
                    const int64_t d = p.g.rowptr[v + 1] - beg;
                    if (d == 0) break;
                    const uint64_t r = draw(key, c0, (uint32_t)s, (uint32_t)v, 0u, (uint64_t)d);
                    const int32_t u = p.g.col[beg + (int64_t)r];
                    if (kMH) {
                        const uint64_t du = (uint64_t)(p.g.rowptr[u + 1] - p.g.rowptr[u]);
                        const uint64_t x = draw(key, c0, (uint32_t)s, (uint32_t)v, 4u, uint64_t(1) << 32);
                        if (x * du < ((uint64_t)d << 32)) v = u;
                    } else {
                        v = u;
                    }
                    path[s + 1] = v;
                }
                for (int64_t q = s + 1; q < L1; ++q) path[q] = -1;
            }
            my_steps = s;
        }
        if (p.batch.req) {  // lanes of one wave may belong to different requests
            if (my_steps) atomicAdd(my_counter, (unsigned long long)my_steps);
        } else {
            const int64_t ws = wave_sum_i64(my_steps);
            if (lane_id() == 0 && ws) atomicAdd(p.steps, (unsigned long long)ws);
        }
    }
}

// is x in the sorted list col[b, e)?
__device__ __forceinline__ bool in_sorted(const int32_t* __restrict__ col, int64_t b, int64_t e, int32_t x) {
    int64_t lo = b, hi = e;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t y = col[mid];
        if (y < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < e && col[lo] == x;
}

// Weighted and node2vec steps: one wavefront per walker. Pass 1 streams
// N(v) in tiles of kWalkTile candidates (kWalkPer coalesced loads per lane,
// the next tile's loads in flight while the current one is processed),
// evaluates the biases and records the inclusive prefix at the end of every
// group of 2^shift tiles in an LDS table (at most kWalkTab groups). After the
// draw, a binary search in the table finds the group and pass 2 rescans only
// that group, 64 candidates at a time (scan + ballot).
// node2vec: x in N(t) is found by merging N(v) with N(t) -- both sorted --
// through an LDS window of kWalkWin entries of N(t) (the following window is
// prefetched into registers), or, when N(t) is much longer than N(v), by a
// binary search per candidate; membership of the first kWalkBits candidates
// is kept as bits for pass 2.
constexpr int kWalkPer = 4;
constexpr int kWalkTile = kWalkPer * kWave;   // 256
constexpr int kWalkTileLog = 8;
constexpr int kWalkTab = 256;
constexpr int kWalkWin = 256;
constexpr int kWinPer = kWalkWin / kWave;
constexpr int kWalkBits = 16384;
constexpr int64_t kMergeRatio = 8;              // merge while d_t <= 8 d_v + kWalkWin

template <bool kN2v>
struct WalkLds {
    uint64_t tab[kWalkTab + 1];
    uint32_t bits[kN2v ? kWalkBits / 32 : 1];
    int32_t win[kN2v ? kWalkWin : 1];
};

// Entries of win[0, kWalkWin) below each of x[0..kWalkPer): four branch-free
// binary searches stepped together, so their LDS reads overlap. The window
// is padded with INT32_MAX; callers use a rank only for x no larger than the
// window's last real entry, where it is the lower bound among the real ones.
__device__ __forceinline__ void win_rank4(const int32_t* win, const int32_t (&x)[kWalkPer], int32_t (&r)[kWalkPer]) {
#pragma unroll
    for (int q = 0; q < kWalkPer; ++q) r[q] = 0;
#pragma unroll
    for (int step = kWalkWin / 2; step >= 1; step >>= 1) {
#pragma unroll
        for (int q = 0; q < kWalkPer; ++q) r[q] += win[r[q] + step - 1] < x[q] ? step : 0;
    }
}

// N(t) window loads: entries [at, at + kWalkWin) of col, clipped to te
__device__ __forceinline__ void load_window(const int32_t* __restrict__ col, int64_t at, int64_t te,
                                            int32_t (&y)[kWinPer]) {
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < kWinPer; ++q) {
        const int64_t i = at + q * kWave + lane;
        y[q] = i < te ? col[i] : INT32_MAX;
    }
}

template <bool kN2v>
__device__ __forceinline__ int64_t walk_step_biased(const WalkParams& p, WalkLds<kN2v>& lds, Key key, uint32_t c0,
                                                    int32_t s, int32_t v, int64_t beg, int64_t d, int32_t t,
                                                    int64_t tb, int64_t te, bool& stop) {
    const int lane = lane_id();
    const int32_t* col = p.g.col;
    const uint32_t* wts = p.bias == kEdgeWeight ? p.g.ew : p.g.degw;
    // pass 1 reads weights (first-order) or neighbor ids (node2vec)
    const uint32_t* src = kN2v ? (const uint32_t*)col + beg : wts + beg;
    stop = false;
    int shift = 0;
    while (((d + ((int64_t)kWalkTile << shift) - 1) >> (kWalkTileLog + shift)) > kWalkTab) ++shift;
    const int64_t g = (int64_t)kWalkTile << shift;
    const int64_t ng = (d + g - 1) / g;
    const bool merge = kN2v && (te - tb) <= kMergeRatio * d + kWalkWin;
    int64_t jw = tb;  // N(t) window: win[0, wn) = col[jw, jw + wn)
    int32_t wn = 0;
    int32_t ynext[kWinPer];
    if (merge) load_window(col, jw, te, ynext);
    uint32_t cur[kWalkPer], nxt[kWalkPer];
#pragma unroll
    for (int q = 0; q < kWalkPer; ++q) {
        const int64_t idx = q * kWave + lane;
        cur[q] = idx < d ? src[idx] : 0u;
    }
    uint64_t run = 0;
    for (int64_t base = 0; base < d; base += kWalkTile) {
#pragma unroll
        for (int q = 0; q < kWalkPer; ++q) {  // next tile in flight
            const int64_t idx = base + kWalkTile + q * kWave + lane;
            nxt[q] = idx < d ? src[idx] : 0u;
        }
        uint32_t x[kWalkPer];
        if (!kN2v) {
#pragma unroll
            for (int q = 0; q < kWalkPer; ++q) x[q] = cur[q];
        } else {
            int32_t a[kWalkPer];
            bool open[kWalkPer], found[kWalkPer];
#pragma unroll
            for (int q = 0; q < kWalkPer; ++q) {
                open[q] = base + q * kWave + lane < d;
                a[q] = (int32_t)cur[q];
                found[q] = false;
            }
            if (merge) {
                while (true) {
                    const int32_t wmax = wn > 0 ? lds.win[wn - 1] : INT32_MIN;
                    bool take[kWalkPer], any = false;
#pragma unroll
                    for (int q = 0; q < kWalkPer; ++q) {
                        take[q] = open[q] && a[q] <= wmax;
                        any |= take[q];
                    }
                    if (ballot(any)) {
                        int32_t r[kWalkPer];
                        win_rank4(lds.win, a, r);
#pragma unroll
                        for (int q = 0; q < kWalkPer; ++q) {
                            if (take[q]) {
                                found[q] = lds.win[r[q]] == a[q];
                                open[q] = false;
                            }
                        }
                    }
                    bool pending = false;
#pragma unroll
                    for (int q = 0; q < kWalkPer; ++q) pending |= open[q];
                    if (ballot(pending) == 0) break;
                    jw += wn;  // every entry of this window is below the open candidates
                    if (jw >= te) break;
                    wn = (int32_t)(te - jw < kWalkWin ? te - jw : kWalkWin);
                    wave_lds_sync();
#pragma unroll
                    for (int q = 0; q < kWinPer; ++q) lds.win[q * kWave + lane] = ynext[q];
                    wave_lds_sync();
                    load_window(col, jw + wn, te, ynext);  // the window after it, in flight
                }
            } else {
#pragma unroll
                for (int q = 0; q < kWalkPer; ++q)
                    if (open[q]) found[q] = in_sorted(col, tb, te, a[q]);
            }
#pragma unroll
            for (int q = 0; q < kWalkPer; ++q) {
                const int64_t idx = base + q * kWave + lane;
                const bool valid = idx < d;
                x[q] = !valid ? 0u : (a[q] == t ? p.w_return : (found[q] ? p.w_common : p.w_outward));
                const uint64_t fm = ballot(valid && found[q]);
                const int64_t i0 = base + q * kWave;
                if (i0 < kWalkBits && lane < 2) lds.bits[i0 / 32 + lane] = (uint32_t)(fm >> (32 * lane));
            }
        }
        uint64_t ls = 0;
#pragma unroll
        for (int q = 0; q < kWalkPer; ++q) ls += x[q];
        run += wave_sum_u64(ls);
        const int64_t tile = base >> kWalkTileLog;
        if (((tile + 1) & ((1ll << shift) - 1)) == 0 || base + kWalkTile >= d)
            if (lane == 0) lds.tab[(tile >> shift) + 1] = run;
#pragma unroll
        for (int q = 0; q < kWalkPer; ++q) cur[q] = nxt[q];
    }
    const uint64_t W = run;
    if (W == 0) {
        stop = true;
        return 0;
    }
    if (lane == 0) lds.tab[0] = 0;
    wave_lds_sync();
    const uint64_t r = draw(key, c0, (uint32_t)s, (uint32_t)v, 0u, W);
    int64_t lo = 0, hi = ng;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (lds.tab[mid] <= r) lo = mid;
        else hi = mid;
    }
    uint64_t acc = lds.tab[lo];
    const int64_t end = (lo + 1) * g < d ? (lo + 1) * g : d;
    int64_t m = end - 1;
    for (int64_t base = lo * g; base < end; base += kWave) {
        const int64_t idx = base + lane;
        uint32_t x = 0;
        if (idx < end) {
            if (!kN2v) {
                x = wts[beg + idx];
            } else {
                const int32_t a = col[beg + idx];
                const bool found = idx < kWalkBits ? ((lds.bits[idx >> 5] >> (idx & 31)) & 1u) != 0
                                                   : in_sorted(col, tb, te, a);
                x = a == t ? p.w_return : (found ? p.w_common : p.w_outward);
            }
        }
        const uint64_t incl = wave_incl_scan_u64(x);
        const uint64_t tot = readlane_u64(incl, kWave - 1);
        if (acc + tot > r) {
            m = base + __popcll(ballot(acc + incl <= r));
            break;
        }
        acc += tot;
    }
    wave_lds_sync();  // the table and bits are rewritten by the next step
    return m;
}

// node2vec step for lists of at most kWalkBits candidates. The bias of x is
// w_return (x = t), w_common (x in N(t)) or w_outward, so the prefix is fixed
// by the membership bits and the position of t: pass 1 only finds membership
// (merge of sorted N(v) with N(t) through the LDS window, a branch-free
// search per candidate), keeping one bit per candidate and their count;
// W = w_out (d - c - [t in N(v)]) + w_common c + w_return [t in N(v)]. Pass 2
// finds the 32-candidate word holding r from word popcounts (64 words per
// ballot) and the candidate inside it.
__device__ __forceinline__ int64_t walk_step_n2v(const WalkParams& p, WalkLds<true>& lds, Key key, uint32_t c0,
                                                 int32_t s, int32_t v, int64_t beg, int64_t d, int32_t t,
                                                 int64_t tb, int64_t te, bool& stop) {
    const int lane = lane_id();
    const int32_t* col = p.g.col;
    stop = false;
    const bool merge = (te - tb) <= kMergeRatio * d + kWalkWin;
    int64_t jw = tb;
    int32_t wn = 0;
    int32_t ynext[kWinPer];
    if (merge) load_window(col, jw, te, ynext);
    int32_t cur[kWalkPer], nxt[kWalkPer];
#pragma unroll
    for (int q = 0; q < kWalkPer; ++q) {
        const int64_t idx = q * kWave + lane;
        cur[q] = idx < d ? col[beg + idx] : 0;
    }
    uint64_t members = 0, nt = 0;  // candidates in N(t) other than t; copies of t
    int64_t pos_t = -1;            // first copy of t (sorted lists keep copies together)
    for (int64_t base = 0; base < d; base += kWalkTile) {
#pragma unroll
        for (int q = 0; q < kWalkPer; ++q) {  // next tile in flight
            const int64_t idx = base + kWalkTile + q * kWave + lane;
            nxt[q] = idx < d ? col[beg + idx] : 0;
        }
        bool open[kWalkPer], found[kWalkPer];
#pragma unroll
        for (int q = 0; q < kWalkPer; ++q) {
            open[q] = base + q * kWave + lane < d;
            found[q] = false;
        }
        if (merge) {
            while (true) {
                const int32_t wmax = wn > 0 ? lds.win[wn - 1] : INT32_MIN;
                bool take[kWalkPer], any = false;
#pragma unroll
                for (int q = 0; q < kWalkPer; ++q) {
                    take[q] = open[q] && cur[q] <= wmax;
                    any |= take[q];
                }
                if (ballot(any)) {
                    int32_t r[kWalkPer];
                    win_rank4(lds.win, cur, r);
#pragma unroll
                    for (int q = 0; q < kWalkPer; ++q) {
                        if (take[q]) {
                            found[q] = lds.win[r[q]] == cur[q];
                            open[q] = false;
                        }
                    }
                }
                bool pending = false;
#pragma unroll
                for (int q = 0; q < kWalkPer; ++q) pending |= open[q];
                if (ballot(pending) == 0) break;
                jw += wn;
                if (jw >= te) break;
                wn = (int32_t)(te - jw < kWalkWin ? te - jw : kWalkWin);
                wave_lds_sync();
#pragma unroll
                for (int q = 0; q < kWinPer; ++q) lds.win[q * kWave + lane] = ynext[q];
                wave_lds_sync();
                load_window(col, jw + wn, te, ynext);
            }
        } else {
#pragma unroll
            for (int q = 0; q < kWalkPer; ++q)
                if (open[q]) found[q] = in_sorted(col, tb, te, cur[q]);
        }
#pragma unroll
        for (int q = 0; q < kWalkPer; ++q) {
            const bool valid = base + q * kWave + lane < d;
            const uint64_t fm = ballot(valid && found[q] && cur[q] != t);
            const uint64_t tm = ballot(valid && cur[q] == t);
            const int64_t i0 = base + q * kWave;
            if (lane < 2) lds.bits[i0 / 32 + lane] = (uint32_t)(fm >> (32 * lane));
            members += __popcll(fm);
            if (tm && pos_t < 0) pos_t = i0 + __ffsll((unsigned long long)tm) - 1;
            nt += __popcll(tm);
            cur[q] = nxt[q];
        }
    }
    const uint64_t wo = p.w_outward, wc = p.w_common, wr = p.w_return;
    const uint64_t W = wo * ((uint64_t)d - members - nt) + wc * members + wr * nt;
    if (W == 0) {
        stop = true;
        return 0;
    }
    wave_lds_sync();
    const uint64_t r = draw(key, c0, (uint32_t)s, (uint32_t)v, 0u, W);
    // S(i) = total bias of candidates [0, i) = wo (i - C - T) + wc C + wr T with
    // C members and T copies of t before i: find the word holding r
    const auto copies_before = [&](int64_t i) -> uint64_t {
        if (pos_t < 0 || i <= pos_t) return 0;
        return (uint64_t)(i - pos_t) < nt ? (uint64_t)(i - pos_t) : nt;
    };
    const int64_t nwords = (d + 31) / 32;
    int64_t wstar = 0;
    uint64_t Cw = 0, prevC = 0;  // members before the chosen word / before the last word of the previous run
    uint32_t carry = 0;
    for (int64_t w0 = 0; w0 < nwords; w0 += kWave) {
        const int64_t w = w0 + lane;
        const bool valid = w < nwords;
        const uint32_t pc = valid ? (uint32_t)__popc(lds.bits[w]) : 0u;
        const uint32_t incl = wave_incl_scan_u32(pc);
        const uint64_t C = (uint64_t)carry + (incl - pc);
        const int64_t i = w * 32;
        const uint64_t T = copies_before(i);
        const uint64_t S = wo * ((uint64_t)i - C - T) + wc * C + wr * T;
        const int nle = __popcll(ballot(valid && S <= r));
        const int nvalid = (int)(nwords - w0 < kWave ? nwords - w0 : kWave);
        if (nle < nvalid || w0 + kWave >= nwords) {  // the word holding r ends here
            if (nle == 0) {  // r starts this run: it is in the last word of the previous one
                wstar = w0 - 1;
                Cw = prevC;
            } else {
                wstar = w0 + nle - 1;
                Cw = readlane_u64(C, nle - 1);
            }
            break;
        }
        prevC = readlane_u64(C, kWave - 1);
        carry += readlane_u32(incl, kWave - 1);
    }
    const int64_t e0 = wstar * 32;
    const uint64_t Tw = copies_before(e0);
    const uint64_t Sw = wo * ((uint64_t)e0 - Cw - Tw) + wc * Cw + wr * Tw;
    const uint32_t word = lds.bits[wstar];
    const int64_t j = e0 + lane;
    uint64_t b = 0;
    if (lane < 32 && j < d)
        b = (pos_t >= 0 && j >= pos_t && (uint64_t)(j - pos_t) < nt) ? wr : (((word >> lane) & 1u) ? wc : wo);
    const uint64_t incl = wave_incl_scan_u64(b);
    const int64_t m = e0 + __popcll(ballot(lane < 32 && j < d && Sw + incl <= r));
    wave_lds_sync();  // bits are rewritten by the next step
    return m;
}

// First-order weighted step on a list of at most kWaveMaxD candidates, in one
// memory round trip: lane i loads candidates i, i + 64, ... of the list,
// weights and neighbor ids together (coalesced). The weights pass through LDS
// so that lane i holds the run [8i, 8i + 8); the lanes' totals are scanned,
// r is drawn in [0, W) and m = #{i : S_(i+1) <= r} (the candidate whose
// interval [S_i, S_(i+1)) holds r) is the number of whole runs below r plus
// the count inside the run that holds it. Returns the neighbor id.
// The step's Philox word on the vector unit. A walk step is wave-uniform, so
// its Philox rounds would otherwise run on the scalar unit (one per compute
// unit), which the step's other uniform work (addresses, loop control)
// already keeps busy; the vector unit forms each 32 x 32 -> 64-bit product in
// one instruction. The same rounds as philox_u64: the empty asm only places
// the counter words in vector registers. The caller takes it at the top of
// the step (the counter is known before any list data arrives) and reduces it
// to [0, W) with range_reduce once W is known.
__device__ __forceinline__ uint64_t philox_vec(Key key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
    uint32_t k0 = key.k0, k1 = key.k1;
    asm volatile("" : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3), "+v"(k0), "+v"(k1));
    return (uint64_t)uniform_i64((int64_t)philox_u64(k0, k1, c0, c1, c2, c3));
}

constexpr int kShortPer = kWaveMaxD / kWave;  // 8
static_assert(sizeof(WalkLds<false>::tab) >= kWaveMaxD * sizeof(uint32_t), "short-list staging fits the LDS table");
__device__ __forceinline__ int32_t walk_step_short(const uint32_t* __restrict__ w, const int32_t* __restrict__ col,
                                                   uint32_t* sh, uint64_t u, int64_t beg, int32_t d, bool& stop) {
    const int lane = lane_id();
    uint32_t x[kShortPer];
    int32_t y[kShortPer];
#pragma unroll
    for (int q = 0; q < kShortPer; ++q) {
        const int32_t i = q * kWave + lane;
        const bool in = i < d;
        x[q] = in ? w[beg + i] : 0u;
        y[q] = in ? col[beg + i] : 0;
    }
#pragma unroll
    for (int q = 0; q < kShortPer; ++q) sh[q * kWave + lane] = x[q];
    wave_lds_sync();
    uint32_t a[kShortPer];
#pragma unroll
    for (int k = 0; k < kShortPer; ++k) a[k] = sh[lane * kShortPer + k];
    wave_lds_sync();  // the next step rewrites sh
    uint64_t t = 0;
#pragma unroll
    for (int k = 0; k < kShortPer; ++k) t += a[k];
    const uint64_t incl = wave_incl_scan_u64(t);
    const uint64_t W = readlane_u64(incl, kWave - 1);
    stop = W == 0;
    if (stop) return -1;
    const uint64_t r = range_reduce(u, W);
    const int L = __popcll(ballot(incl <= r));  // whole runs below r: lane L's run holds it
    uint64_t acc = incl - t;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kShortPer; ++k) {
        acc += a[k];
        c += acc <= r ? 1u : 0u;
    }
    const int32_t m = L * kShortPer + (int32_t)readlane_u32(c, L);
    const int qm = m / kWave;
    int32_t nb = y[0];
#pragma unroll
    for (int q = 1; q < kShortPer; ++q) nb = q == qm ? y[q] : nb;
    return readlane_i32(nb, m % kWave);
}

// First-order weighted step on a list longer than kWaveMaxD, through the
// graph's tables instead of a pass over the list: ctab holds the list's
// running total at the end of each 1024-weight chunk (so W is its last
// entry), gtab each chunk's inclusive 16-weight group prefixes. The chunk
// holding r is found by ballot over up to 64 running totals (lists of more
// than 64 chunks first narrow the range with 64 evenly spaced totals), the
// group by ballot over the chunk's 64 group prefixes, and the candidate from
// the group's 16 weights, loaded with their neighbor ids. Every sum is exact,
// so the pick is the one a scan of the whole list gives. Returns the neighbor.
constexpr int kWalkTotLoads = 4;  // lists of up to 4 * 64 chunks read every running total at once
__device__ __forceinline__ int32_t walk_step_long(const uint32_t* __restrict__ w, const int32_t* __restrict__ col,
                                                  const uint64_t* __restrict__ gtab,
                                                  const uint64_t* __restrict__ ctab, uint64_t u, int64_t beg, int64_t d,
                                                  bool& stop) {
    const int lane = lane_id();
    const int64_t row0 = beg >> kTabShift;
    const uint64_t* C = ctab + row0;
    const int64_t nch = (d + kChunk - 1) / kChunk;
    int64_t lo = 0, hi = nch;  // r lies in chunks [lo, hi)
    uint64_t acc = 0;          // running total before chunk lo
    uint64_t r = 0;
    bool drawn = false;
    int64_t j = 0;
    if (nch <= (int64_t)kWave * kWalkTotLoads) {
        // every running total at once: lane L holds totals q * 64 + L, all
        // loads issued before any is used (one memory round trip); j is the
        // number of totals at or below r (they never decrease)
        uint64_t e[kWalkTotLoads];
#pragma unroll
        for (int q = 0; q < kWalkTotLoads; ++q) {
            const int64_t i = (int64_t)q * kWave + lane;
            e[q] = ~0ull;
            if ((int64_t)q * kWave < nch && i < nch) e[q] = C[i];
        }
        const int64_t last = nch - 1;
        uint64_t el = e[0];
#pragma unroll
        for (int q = 1; q < kWalkTotLoads; ++q) el = q == (int)(last / kWave) ? e[q] : el;
        const uint64_t W = readlane_u64(el, (int)(last % kWave));  // total of the whole list
        stop = W == 0;
        if (stop) return -1;
        r = range_reduce(u, W);
        int64_t c = 0;
#pragma unroll
        for (int q = 0; q < kWalkTotLoads; ++q) c += __popcll(ballot(e[q] <= r));
        j = c;
        if (c > 0) {
            uint64_t ec = e[0];
#pragma unroll
            for (int q = 1; q < kWalkTotLoads; ++q) ec = q == (int)((c - 1) / kWave) ? e[q] : ec;
            acc = readlane_u64(ec, (int)((c - 1) % kWave));
        }
        lo = hi;  // done: skip the sampled search below
    }
    while (lo < hi) {
        const int64_t len = hi - lo;
        const int64_t stride = (len + kWave - 1) / kWave;
        const int64_t nb = (len + stride - 1) / stride;  // sampled totals (lanes in use)
        const bool in = lane < nb;
        int64_t idx = lo + (int64_t)(lane + 1) * stride - 1;
        idx = idx < hi ? idx : hi - 1;
        const uint64_t e = in ? C[idx] : ~0ull;
        if (!drawn) {
            const uint64_t W = readlane_u64(e, (int)nb - 1);  // total of the whole list
            stop = W == 0;
            if (stop) return -1;
            r = range_reduce(u, W);
            drawn = true;
        }
        const int c = __popcll(ballot(in && e <= r));  // sampled ranges ending at or below r
        if (c > 0) acc = readlane_u64(e, c - 1);
        if (stride == 1) {
            j = lo + c;
            break;
        }
        lo += (int64_t)c * stride;
        hi = lo + stride < hi ? lo + stride : hi;
    }
    const uint64_t gp = gtab[(row0 + j) * kChunkGroups + lane];  // inclusive prefix of groups 0..lane of chunk j
    const int gi = __popcll(ballot(acc + gp <= r));              // the group holding r
    const uint64_t before = acc + (gi > 0 ? readlane_u64(gp, gi - 1) : 0ull);
    const int64_t i0 = j * kChunk + (int64_t)gi * 16;
    const bool in = lane < 16 && i0 + lane < d;
    // the group's weights and ids at clamped positions, lanes past it zeroed
    const int64_t ii = beg + (in ? i0 + lane : i0);
    uint64_t x = (uint64_t)w[ii];
    const int32_t y = col[ii];
    x = in ? x : 0ull;
    const uint64_t incl = wave_incl_scan_u64(x);
    const int k = __popcll(ballot(in && before + incl <= r));
    return readlane_i32(y, k);
}

// First-order weighted step on a list longer than kWaveMaxD through its walk
// guide, one wavefront per walker: r is drawn in [0, W) (W, the list's total,
// came with the row offsets), its bucket k = r >> s gives the bracket
// [G[k], G[k+1]] that holds the pick (every position before G[k] ends at or
// below k * 2^s <= r, and G[k+1] ends past (k+1) * 2^s > r), and one load of
// the bracket's exact prefixes and neighbor ids finds m = #{i : S_(i+1) <= r}
// by ballot. Three dependent loads per step (row offsets and W, the bracket,
// its prefixes), two when the bracket holds one or two positions (the
// buckets carry their positions' prefixes and ids). Returns the neighbor,
// or -2 when the bracket is wider than a
// wavefront (many small weights in one bucket), which the caller takes
// through the chunk tables.
__device__ __forceinline__ int32_t walk_step_guide(const WalkEdge* __restrict__ er,
                                                   const WalkBucket* __restrict__ gd, uint64_t r, uint64_t W,
                                                   int64_t beg, int64_t d, int64_t v) {
    const int lane = lane_id();
    const int sh = guide_shift(W, d);
    const uint64_t K = ((W - 1) >> sh) + 1;
    const uint64_t k = r >> sh;
    const WalkBucket* G = gd + guide_base(beg, v);
    const bool last = k + 1 >= K;
    const WalkBucket* q0 = G + k;
    const WalkBucket* q1 = G + (last ? k : k + 1);
    const WalkBucket b0{ld_uniform(&q0->S), ld_uniform(&q0->pos), ld_uniform(&q0->col)};
    const WalkBucket b1{ld_uniform(&q1->S), ld_uniform(&q1->pos), ld_uniform(&q1->col)};
    const int64_t lo = b0.pos;
    const int64_t hi = last ? d - 1 : (int64_t)b1.pos;
    // a bracket of one or two positions: the buckets hold their prefixes and ids
    if (hi == lo) return b0.col;
    if (!last && hi == lo + 1) return b0.S > r ? b0.col : b1.col;
    const int64_t n = hi - lo + 1;
    if (n > kWave) return -2;
    // both loads issued at clamped positions, then the lanes past the
    // bracket masked: guarded loads were waited for one after the other
    const bool in = lane < n;
    const int64_t j = beg + lo + (in ? lane : n - 1);
    uint64_t S = er[j].S;
    const int32_t y = er[j].col;
    __builtin_amdgcn_sched_barrier(0);  // both loads in flight before either is used
    S = in ? S : ~0ull;
    const int c = __popcll(ballot(S <= r));
    return readlane_i32(y, c);
}

// node2vec step from v when the previous vertex t has a short list (fewer
// than 64 entries) and N(v) a long one: instead of merging all of N(v) with
// N(t), lane k takes the k-th entry x of N(t) and binary-searches both ends
// of x's run in N(v) (lane d_t does the same for t itself), so membership
// costs about log2(d_v) dependent loads whatever d_v is. The pick is found
// without reading N(v) again: with C(j) = common candidates below position j
// (a wave sum over the lanes' runs; a repeated x counts once) and T(j) =
// copies of t below j, the exclusive prefix is
// S(j) = w_out (j - C - T) + w_common C + w_return T, and m is the smallest i
// with S(i + 1) > r, by binary search over i: the same m as the merge.
constexpr int64_t kShortPrevMinD = 2048;  // shorter N(v): the merge is cheaper
__device__ __forceinline__ int64_t walk_step_n2v_short_prev(const WalkParams& p, Key key, uint32_t c0, int32_t s,
                                                            int32_t v, int64_t beg, int64_t d, int32_t t,
                                                            int64_t tb, int64_t te, bool& stop) {
    const int lane = lane_id();
    const int32_t* __restrict__ col = p.g.col;
    const int64_t dt = te - tb;  // < kWave
    const bool act = lane <= dt;
    const int32_t x = lane < dt ? col[tb + lane] : t;
    // [lo1, lo2): the run of x in N(v) (lower and upper bound, side by side)
    int64_t lo1 = 0, hi1 = act ? d : 0, lo2 = 0, hi2 = act ? d : 0;
    while (ballot(lo1 < hi1 || lo2 < hi2)) {
        const bool s1 = lo1 < hi1, s2 = lo2 < hi2;
        const int64_t m1 = (lo1 + hi1) >> 1, m2 = (lo2 + hi2) >> 1;
        const int32_t y1 = col[beg + (s1 ? m1 : 0)];
        const int32_t y2 = col[beg + (s2 ? m2 : 0)];
        if (s1) {
            if (y1 < x) lo1 = m1 + 1;
            else hi1 = m1;
        }
        if (s2) {
            if (y2 <= x) lo2 = m2 + 1;
            else hi2 = m2;
        }
    }
    const int32_t xprev = __shfl_up(x, 1, kWave);
    const bool common = lane < dt && (lane == 0 || xprev != x) && x != t && lo2 > lo1;
    const int64_t cnt = lo2 - lo1;
    const int64_t pos_t = readlane_i64(lo1, (int)dt);
    const int64_t n_t = readlane_i64(lo2, (int)dt) - pos_t;
    const uint64_t c = (uint64_t)wave_sum_i64(common ? cnt : 0);
    const uint64_t wo = p.w_outward, wc = p.w_common, wr = p.w_return;
    const uint64_t W = wo * ((uint64_t)d - c - (uint64_t)n_t) + wc * c + wr * (uint64_t)n_t;
    stop = W == 0;
    if (stop) return 0;
    const uint64_t r = draw(key, c0, (uint32_t)s, (uint32_t)v, 0u, W);
    int64_t a = 0, b = d - 1;  // S(d) = W > r
    while (a < b) {
        const int64_t mid = (a + b) >> 1, j = mid + 1;
        const int64_t below = j - lo1 < 0 ? 0 : (j - lo1 < cnt ? j - lo1 : cnt);
        const uint64_t C = (uint64_t)wave_sum_i64(common ? below : 0);
        const uint64_t T = j <= pos_t ? 0 : (uint64_t)(j - pos_t < n_t ? j - pos_t : n_t);
        const uint64_t S = wo * ((uint64_t)j - C - T) + wc * C + wr * T;
        if (S > r) b = mid;
        else a = mid + 1;
    }
    return a;
}

template <bool kN2v, bool kMoves>
__device__ __forceinline__ void walk_wave_body(const WalkParams& p) {
    __shared__ WalkLds<kN2v> lds_all[kWavesPerBlock];
    const int lane = lane_id();
    const int wid = uniform_i32(threadIdx.x / kWave);
    WalkLds<kN2v>& lds = lds_all[wid];
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t w = blockIdx.x * (int64_t)kWavesPerBlock + wid; w < p.num_walkers; w += waves) {
        const WalkerCtx wc = walker_ctx(p, w);
        const Key key{(uint32_t)uniform_i32((int32_t)wc.key.k0), (uint32_t)uniform_i32((int32_t)wc.key.k1)};
        const int32_t length = uniform_i32(wc.length);
        const int64_t L1 = (int64_t)length + 1;
        int32_t* path = wc.path;
        int32_t v = uniform_i32(p.starts[w]);
        if (v < 0 || (int64_t)v >= p.g.n) {
            if (lane == 0) *p.bad_start = 1;
            for (int64_t q = lane; q < L1; q += kWave) path[q] = -1;
            continue;
        }
        if (lane == 0) path[0] = v;
        const uint32_t c0 = (uint32_t)uniform_i32((int32_t)wc.c0);
        const int32_t start = v;
        int32_t t = -1;
        int64_t tb = 0, te = 0;
        int32_t s = 0;
        for (; s < length; ++s) {
            int32_t to;
            if (kMoves && walk_move(p, key, c0, s, v, start, to)) {  // uniform: the draw depends on wave-uniform values
                if (lane == 0) path[s + 1] = to;
                v = to;
                t = -1;
                tb = te = 0;
                continue;
            }
            int64_t beg, d;
            row_uniform(p.g.rowptr, v, beg, d);
            // first-order steps: the list's total (for the walk guide) with the
            // row offsets, and the draw's Philox word while they load
            uint64_t u = 0, wt = 0;
            if constexpr (!kN2v) {
                const bool dg = p.bias == kNeighborDegree;
                const uint64_t* tots = dg ? p.g.wtot_deg : p.g.wtot_ew;
                if ((dg ? p.g.wgd_deg : p.g.wgd_ew) != nullptr) wt = ld_uniform(tots + v);
                u = philox_vec(key, c0, (uint32_t)s, (uint32_t)v, 0u);
            }
            if (d == 0) break;
            int64_t m = -1;  // position of the pick (paths that return the neighbor itself leave -1)
            int32_t nx = -1;
            bool stop = false;
            if (kN2v && t < 0) {  // first step: no previous vertex, every bias is 1
                m = (int64_t)draw(key, c0, (uint32_t)s, (uint32_t)v, 0u, (uint64_t)d);
            } else {
                if constexpr (kN2v) {
                    if (te - tb < kWave && d >= kShortPrevMinD)
                        m = walk_step_n2v_short_prev(p, key, c0, s, v, beg, d, t, tb, te, stop);
                    else if (d <= kWalkBits) m = walk_step_n2v(p, lds, key, c0, s, v, beg, d, t, tb, te, stop);
                    else m = walk_step_biased<true>(p, lds, key, c0, s, v, beg, d, t, tb, te, stop);
                } else {
                    const bool dg = p.bias == kNeighborDegree;
                    const uint32_t* wts = dg ? p.g.degw : p.g.ew;
                    const uint64_t* gt = dg ? p.g.gtab_deg : p.g.gtab_ew;
                    const uint64_t* ct = dg ? p.g.ctab_deg : p.g.ctab_ew;
                    const WalkEdge* er = dg ? p.g.wrec_deg : p.g.wrec_ew;
                    const WalkBucket* gd = dg ? p.g.wgd_deg : p.g.wgd_ew;
                    if (d <= kWaveMaxD || (gt && ct)) {
                        if (d <= kWaveMaxD) {
                            nx = walk_step_short(wts, p.g.col, reinterpret_cast<uint32_t*>(lds.tab), u, beg, (int32_t)d,
                                                 stop);
                        } else {
                            nx = -2;
                            if (gd) {
                                stop = wt == 0;
                                if (!stop) nx = walk_step_guide(er, gd, range_reduce(u, wt), wt, beg, d, v);
                            }
                            if (nx == -2 && !stop) nx = walk_step_long(wts, p.g.col, gt, ct, u, beg, d, stop);
                        }
                    } else {
                        m = walk_step_biased<false>(p, lds, key, c0, s, v, beg, d, t, tb, te, stop);
                    }
                }
                if (stop) break;
            }
            if (m >= 0) nx = ld_uniform(p.g.col + beg + m);
            nx = uniform_i32(nx);
            if (lane == 0) path[s + 1] = nx;
            t = v;
            tb = beg;
            te = beg + d;
            v = nx;
        }
        for (int64_t q = s + 1 + lane; q < L1; q += kWave) path[q] = -1;
        if (lane == 0 && s) atomicAdd(wc.steps, (unsigned long long)s);
    }
}

// First-order walks are bound by the latency of their dependent loads, so
// they are held to 8 waves per SIMD (the scalar registers this needs spill
// to vector lanes, not to memory); walks with restart / jump moves and
// node2vec keep their larger register sets.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) k_walk_wave_first(WalkParams p) {
    walk_wave_body<false, false>(p);
}

__global__ void __launch_bounds__(kBlock) k_walk_wave_moves(WalkParams p) {
    walk_wave_body<false, true>(p);
}

template <bool kMoves>
__global__ void __launch_bounds__(kBlock) k_walk_wave_n2v(WalkParams p) {
    walk_wave_body<true, kMoves>(p);
}

// Weighted first-order walks through the walk guide, one lane per walker
// (64 walkers per wavefront, each with its own chain of loads). A step:
// the vertex's record, its list and total W (one 16-byte load; the Philox
// word is formed meanwhile), r = floor(u W / 2^64), the bracket
// [G[k], G[k+1]] of bucket k = r >> s (one load of two 16-byte buckets; a
// bracket of one or two positions is decided by the buckets' own prefixes
// and ids, about 80% of steps), else the edge records of the bracket's first
// kLaneProbe positions, exact prefixes beside neighbor ids (one round):
// m = lo + #{j : S_(lo+j+1) <= r}. The walk is bound by the 128-byte lines
// these scattered reads pull from HBM, so each round reads one line where
// it can. Positions
// past the bracket's end are read at the end instead, whose prefix exceeds r,
// so every load stays inside the list and needs no mask. A bracket longer
// than the probe (rare: a run of small weights inside one bucket) takes
// further rounds from where the last one stopped. A list of one edge skips
// the bracket. The pick is the same m as a scan of the whole list.
constexpr int kLaneProbe = 8;
// A lane's round waits for the slowest of its wavefront's 64 scattered
// loads, so an unloaded lane step takes longer than a wavefront step (3.3
// against 2.0 us at 2,048 walkers); the lane kernel wins once a launch has
// enough walkers to keep many lanes' chains in flight (measured: behind at
// 8,192 walkers, ahead at 16,384).
constexpr int64_t kLaneWalkMin = 12288;

// A lane's path entries, written kPathRun at a time: a 4-byte store into a row
// of its own per step leaves each line part written in the L2 when it is
// evicted, over and over; a run of consecutive entries reaches its line at
// once.
constexpr int kPathRun = 8;
struct PathRun {
    int32_t e[kPathRun] = {};
    int n = 0;
    int64_t at = 1;  // path index of e[0]
    __device__ __forceinline__ void flush(int32_t* path) {
#pragma unroll
        for (int j = 0; j < kPathRun; ++j)
            if (j < n) path[at + j] = e[j];
        at += n;
        n = 0;
    }
    __device__ __forceinline__ void push(int32_t* path, int32_t x) {
#pragma unroll
        for (int j = 0; j < kPathRun; ++j) e[j] = n == j ? x : e[j];
        if (++n == kPathRun) flush(path);
    }
};

template <bool kMoves>
__global__ void __launch_bounds__(kBlock) k_walk_lane(WalkParams p) {
    const bool dg = p.bias == kNeighborDegree;
    const WalkVertex* __restrict__ vt = dg ? p.g.wvtx_deg : p.g.wvtx_ew;
    const WalkEdge* __restrict__ er = dg ? p.g.wrec_deg : p.g.wrec_ew;
    const WalkBucket* __restrict__ gd = dg ? p.g.wgd_deg : p.g.wgd_ew;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w0 = blockIdx.x * (int64_t)blockDim.x; w0 < p.num_walkers; w0 += stride) {
        const int64_t w = w0 + threadIdx.x;
        int64_t my_steps = 0;
        unsigned long long* my_counter = p.steps;
        if (w < p.num_walkers) {
            const WalkerCtx wc = walker_ctx(p, w);
            const Key key = wc.key;
            const int64_t L1 = (int64_t)wc.length + 1;
            int32_t* path = wc.path;
            my_counter = wc.steps;
            int32_t v = p.starts[w];
            int32_t s = 0;
            if (v < 0 || (int64_t)v >= p.g.n) {
                *p.bad_start = 1;
                for (int64_t q = 0; q < L1; ++q) path[q] = -1;
            } else {
                path[0] = v;
                const int32_t start = v;
                const uint32_t c0 = wc.c0;
                PathRun run;
                for (; s < wc.length; ++s) {
                    int32_t to;
                    if (kMoves && walk_move(p, key, c0, s, v, start, to)) {
                        v = to;
                        run.push(path, v);
                        continue;
                    }
                    const WalkVertex x = vt[v];
                    const int64_t beg = x.beg, d = x.d;
                    const uint64_t W = x.W;
                    uint64_t u = philox_u64(key.k0, key.k1, c0, (uint32_t)s, (uint32_t)v, 0u);
                    // formed while the offsets load, not sunk past the test below
                    asm volatile("" : "+v"(u));
                    if (d == 0 || W == 0) break;
                    const uint64_t r = range_reduce(u, W);
                    int64_t lo = 0, hi = 0;
                    int32_t nx = -1;
                    bool done = false;
                    if (d > 1) {
                        const int sh = guide_shift(W, d);
                        const uint64_t K = ((W - 1) >> sh) + 1;
                        const uint64_t k = r >> sh;
                        const WalkBucket* G = gd + guide_base(beg, v);
                        const bool last = k + 1 >= K;
                        const WalkBucket b0 = G[k], b1 = G[last ? k : k + 1];
                        lo = b0.pos;
                        hi = last ? d - 1 : (int64_t)b1.pos;
                        // a bracket of one or two positions needs no edge record
                        if (hi == lo) {
                            nx = b0.col;
                            done = true;
                        } else if (!last && hi == lo + 1) {
                            nx = b0.S > r ? b0.col : b1.col;
                            done = true;
                        }
                    }
                    while (!done) {
                        uint64_t S[kLaneProbe - 1];
                        int32_t y[kLaneProbe];
#pragma unroll
                        for (int j = 0; j < kLaneProbe; ++j) {
                            const int64_t q = beg + (lo + j < hi ? lo + j : hi);
                            if (j < kLaneProbe - 1) S[j] = er[q].S;
                            y[j] = er[q].col;
                        }
                        int c = 0;
#pragma unroll
                        for (int j = 0; j < kLaneProbe - 1; ++j) c += S[j] <= r ? 1 : 0;
                        nx = y[0];
#pragma unroll
                        for (int j = 1; j < kLaneProbe; ++j) nx = c == j ? y[j] : nx;
                        // keeps the id loads in this round: left to itself the
                        // compiler sinks them past the loop, a round of their own
                        asm volatile("" ::"v"(nx));
                        if (c < kLaneProbe - 1 || lo + kLaneProbe - 1 >= hi) break;
                        lo += kLaneProbe - 1;
                    }
                    v = nx;
                    run.push(path, v);
                }
                run.flush(path);
                for (int64_t q = s + 1; q < L1; ++q) path[q] = -1;
            }
            my_steps = s;
        }
        if (p.batch.req) {  // lanes of one wave may belong to different requests
            if (my_steps) atomicAdd(my_counter, (unsigned long long)my_steps);
        } else {
            const int64_t ws = wave_sum_i64(my_steps);
            if (lane_id() == 0 && ws) atomicAdd(p.steps, (unsigned long long)ws);
        }
    }
}

// One wavefront per vertex u, a lane per edge (u, x): is u in the sorted N(x)?
__global__ void __launch_bounds__(kBlock) k_symmetric_check(RowPtr rowptr, const int32_t* __restrict__ col,
                                                            int64_t n, int32_t* __restrict__ flag) {
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t u = blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave; u < n; u += waves) {
        const int64_t b = rowptr[u], e = rowptr[u + 1];
        bool missing = false;
        for (int64_t i = b + lane; i < e; i += kWave) {
            const int32_t x = col[i];
            missing |= !in_sorted(col, rowptr[x], rowptr[x + 1], (int32_t)u);
        }
        if (ballot(missing) && lane == 0) atomicOr(flag, 1);
    }
}

// Walk guide tables, one wavefront per list with a positive total: the inclusive prefix of every edge (64 at a time, one
// scan each, carried), and for each bucket k < K of the list's guide the
// position i whose interval [S_i, S_(i+1)) holds k * 2^s. Edge i covers the
// buckets from ceil(S_i / 2^s) to ceil(S_(i+1) / 2^s) - 1 (none for a zero
// weight), so every bucket is written once. A lane writes up to
// kGuideLaneFill buckets itself; an edge heavier than that many buckets is
// written by the whole wavefront, 64 buckets at a time.
constexpr uint64_t kGuideLaneFill = 8;
__global__ void __launch_bounds__(kBlock) k_walk_guides(RowPtr rowptr, const int32_t* __restrict__ col,
                                                        const uint32_t* __restrict__ w,
                                                        const uint64_t* __restrict__ wtot, int64_t n,
                                                        WalkEdge* __restrict__ rec, WalkVertex* __restrict__ vtx,
                                                        WalkBucket* __restrict__ gd) {
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t v = blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave; v < n; v += waves) {
        int64_t b, d;
        row_uniform(rowptr, v, b, d);
        const uint64_t W = ld_uniform(wtot + v);
        if (vtx && lane == 0) vtx[v] = WalkVertex{W, (uint32_t)b, (uint32_t)d};
        if (W == 0) continue;
        const int sh = guide_shift(W, d);
        const uint64_t K = ((W - 1) >> sh) + 1;
        const uint64_t low = (uint64_t(1) << sh) - 1;
        WalkBucket* G = gd + guide_base(b, v);
        uint64_t run = 0;
        for (int64_t base = 0; base < d; base += kWave) {
            const int64_t i = base + lane;
            const uint64_t x = i < d ? (uint64_t)w[b + i] : 0ull;
            const int32_t y = i < d ? col[b + i] : 0;
            const uint64_t incl = run + wave_incl_scan_u64(x);
            const uint64_t excl = incl - x;
            const uint64_t k0 = (excl >> sh) + ((excl & low) != 0);
            uint64_t k1 = (incl >> sh) + ((incl & low) != 0);
            k1 = k1 < K ? k1 : K;
            const uint64_t nk = i < d && k1 > k0 ? k1 - k0 : 0;
            if (i < d) {
                rec[b + i] = WalkEdge{incl, y, (uint32_t)x};
                if (nk <= kGuideLaneFill)
                    for (uint64_t k = k0; k < k1; ++k) G[k] = WalkBucket{incl, (uint32_t)i, y};
            }
            for (uint64_t wide = ballot(nk > kGuideLaneFill); wide; wide &= wide - 1) {
                const int src = __ffsll((unsigned long long)wide) - 1;
                const uint64_t a0 = readlane_u64(k0, src), a1 = readlane_u64(k1, src);
                const WalkBucket e{readlane_u64(incl, src), (uint32_t)(base + src), readlane_i32(y, src)};
                for (uint64_t k = a0 + lane; k < a1; k += kWave) G[k] = e;
            }
            run = readlane_u64(incl, kWave - 1);
        }
    }
}

}  // namespace

void launch_walk_guides(RowPtr rowptr, const int32_t* col, const uint32_t* w, const uint64_t* wtot, int64_t n,
                        WalkEdge* rec, WalkVertex* vtx, WalkBucket* gd, hipStream_t s) {
    if (n <= 0) return;
    int64_t g = (n + kWavesPerBlock - 1) / kWavesPerBlock;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_walk_guides, dim3((unsigned)g), dim3(kBlock), 0, s, rowptr, col, w, wtot, n, rec, vtx, gd);
}

void launch_symmetric_check(RowPtr rowptr, const int32_t* col, int64_t n, int32_t* flag, hipStream_t s) {
    if (n <= 0) return;
    int64_t g = (n + kWavesPerBlock - 1) / kWavesPerBlock;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_symmetric_check, dim3((unsigned)g), dim3(kBlock), 0, s, rowptr, col, n, flag);
}

void launch_walk(const WalkParams& p, int grid, hipStream_t s, LaunchEvents ev) {
    if (p.num_walkers <= 0) return;
    const bool flat_n2v = p.bias == kNode2vec && p.w_return == p.w_common && p.w_common == p.w_outward &&
                          p.w_return > 0;
    if (p.bias == kUniform || flat_n2v || p.bias == kMetropolis) {
        int64_t g = (p.num_walkers + kBlock - 1) / kBlock;
        if (g > grid) g = grid;
        if (p.bias == kMetropolis) launch_kernel(k_walk_uniform<true>, dim3((unsigned)g), dim3(kBlock), s, ev, p);
        else launch_kernel(k_walk_uniform<false>, dim3((unsigned)g), dim3(kBlock), s, ev, p);
    } else {
        int64_t g = (p.num_walkers + kWavesPerBlock - 1) / kWavesPerBlock;
        if (g > grid) g = grid;
        const bool moves = (p.restart | p.jump) != 0;
        if (p.bias == kNode2vec) {
            if (moves) launch_kernel(k_walk_wave_n2v<true>, dim3((unsigned)g), dim3(kBlock), s, ev, p);
            else launch_kernel(k_walk_wave_n2v<false>, dim3((unsigned)g), dim3(kBlock), s, ev, p);
        } else {
            const bool dg = p.bias == kNeighborDegree;
            if ((dg ? p.g.wgd_deg : p.g.wgd_ew) && (dg ? p.g.wrec_deg : p.g.wrec_ew) &&
                (dg ? p.g.wvtx_deg : p.g.wvtx_ew) && p.num_walkers >= kLaneWalkMin) {
                int64_t gl = (p.num_walkers + kBlock - 1) / kBlock;
                if (gl > grid) gl = grid;
                if (moves) launch_kernel(k_walk_lane<true>, dim3((unsigned)gl), dim3(kBlock), s, ev, p);
                else launch_kernel(k_walk_lane<false>, dim3((unsigned)gl), dim3(kBlock), s, ev, p);
            } else if (moves) {
                launch_kernel(k_walk_wave_moves, dim3((unsigned)g), dim3(kBlock), s, ev, p);
            } else {
                launch_kernel(k_walk_wave_first, dim3((unsigned)g), dim3(kBlock), s, ev, p);
            }
        }
    }
}

}  // namespace csaw
