// walk_kernels.hip -- gfx950 kernels of random walks (DeepWalk, biased
// DeepWalk, node2vec; Section II-A of the paper).
//
// A walk is a chain of one-draw selections (NeighborSize 1, with
// replacement). The step loop runs inside the kernel: walkers are
// independent, so no host round trip is needed between steps.
//   - unbiased walks: one lane per walker (a step is two row-offset loads,
//     one Philox draw and one neighbor load);
//   - biased walks: one wavefront per walker; the wave sums the biases of
//     N(v) (pass 1), draws r in [0, W), and finds the owning candidate with
//     chunked inclusive scans and a ballot (pass 2). Biases of the first
//     kCache*64 neighbors stay in registers between the passes.
//   - node2vec: the bias of x in N(v) needs "is x adjacent to the previous
//     vertex t"; adjacency lists are sorted, so each lane binary-searches
//     N(t).
#include "device_common.h"
#include "kernels.h"

namespace csaw {

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kCache = 4;  // register-cached 64-wide chunks per lane

__global__ void __launch_bounds__(kBlock) k_walk_uniform(WalkParams p) {
    const Key key{p.k0, p.k1};
    const int64_t L1 = (int64_t)p.length + 1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w0 = blockIdx.x * (int64_t)blockDim.x; w0 < p.num_walkers; w0 += stride) {
        const int64_t w = w0 + threadIdx.x;
        int64_t my_steps = 0;
        if (w < p.num_walkers) {
            int32_t* path = p.paths + w * L1;
            int32_t v = p.starts[w];
            int32_t s = 0;
            if (v < 0 || (int64_t)v >= p.g.n) {
                *p.bad_start = 1;
                for (int64_t q = 0; q < L1; ++q) path[q] = -1;
            } else {
                path[0] = v;
                const uint32_t c0 = (uint32_t)(p.walker_ids ? p.walker_ids[w] : p.walker_base + (uint64_t)w);
                for (; s < p.length; ++s) {
                    const int64_t beg = p.g.rowptr[v];
                    const int64_t d = p.g.rowptr[v + 1] - beg;
                    if (d == 0) break;
                    const uint64_t r = draw(key, c0, (uint32_t)s, (uint32_t)v, 0u, (uint64_t)d);
                    v = p.g.col[beg + (int64_t)r];
                    path[s + 1] = v;
                }
                for (int64_t q = s + 1; q < L1; ++q) path[q] = -1;
            }
            my_steps = s;
        }
        const int64_t ws = wave_sum_i64(my_steps);
        if (lane_id() == 0 && ws) atomicAdd(p.steps, (unsigned long long)ws);
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

struct StepBias {
    int32_t kind;
    const uint32_t* w;
    const int32_t* col;
    uint32_t wr, wc, wo;
    int32_t t;         // previous vertex, -1 before the first step
    int64_t tb, te;    // its list
};

__device__ __forceinline__ uint32_t bias_of(const StepBias& sb, int64_t e) {
    if (sb.kind == kNode2vec) {
        if (sb.t < 0) return 1u;
        const int32_t x = sb.col[e];
        if (x == sb.t) return sb.wr;
        return in_sorted(sb.col, sb.tb, sb.te, x) ? sb.wc : sb.wo;
    }
    return sb.w[e];
}

__global__ void __launch_bounds__(kBlock) k_walk_wave(WalkParams p) {
    const int lane = lane_id();
    const int wid = uniform_i32(threadIdx.x / kWave);
    const Key key{p.k0, p.k1};
    const int64_t L1 = (int64_t)p.length + 1;
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    StepBias sb;
    sb.kind = p.bias;
    sb.w = p.bias == kEdgeWeight ? p.g.ew : p.g.degw;
    sb.col = p.g.col;
    sb.wr = p.w_return;
    sb.wc = p.w_common;
    sb.wo = p.w_outward;
    for (int64_t w = blockIdx.x * (int64_t)kWavesPerBlock + wid; w < p.num_walkers; w += waves) {
        int32_t* path = p.paths + w * L1;
        int32_t v = uniform_i32(p.starts[w]);
        if (v < 0 || (int64_t)v >= p.g.n) {
            if (lane == 0) *p.bad_start = 1;
            for (int64_t q = lane; q < L1; q += kWave) path[q] = -1;
            continue;
        }
        if (lane == 0) path[0] = v;
        const uint32_t c0 = (uint32_t)(p.walker_ids ? p.walker_ids[w] : p.walker_base + (uint64_t)w);
        sb.t = -1;
        sb.tb = sb.te = 0;
        int32_t s = 0;
        for (; s < p.length; ++s) {
            const int64_t beg = uniform_i64(p.g.rowptr[v]);
            const int64_t d = uniform_i64(p.g.rowptr[v + 1]) - beg;
            if (d == 0) break;
            // pass 1: total bias (first kCache chunks kept in registers)
            uint32_t cache[kCache];
            uint64_t part = 0;
#pragma unroll
            for (int c = 0; c < kCache; ++c) {
                const int64_t idx = (int64_t)c * kWave + lane;
                cache[c] = idx < d ? bias_of(sb, beg + idx) : 0u;
                part += cache[c];
            }
            for (int64_t idx = (int64_t)kCache * kWave + lane; idx < d; idx += kWave) part += bias_of(sb, beg + idx);
            const uint64_t W = wave_sum_u64(part);
            if (W == 0) break;
            const uint64_t r = draw(key, c0, (uint32_t)s, (uint32_t)v, 0u, W);
            // pass 2: first chunk whose inclusive prefix passes r
            uint64_t acc = 0;
            int64_t m = 0;
            for (int64_t base = 0; base < d; base += kWave) {
                const int64_t idx = base + lane;
                const int64_t c = base / kWave;
                uint32_t x;
                if (c < kCache) {
                    x = cache[0];
#pragma unroll
                    for (int q = 1; q < kCache; ++q)
                        if (c == q) x = cache[q];
                } else {
                    x = idx < d ? bias_of(sb, beg + idx) : 0u;
                }
                const uint64_t incl = wave_incl_scan_u64(x);
                const uint64_t tot = readlane_u64(incl, kWave - 1);
                if (acc + tot > r) {
                    m = base + __popcll(ballot(acc + incl <= r));
                    break;
                }
                acc += tot;
            }
            const int32_t nx = uniform_i32(p.g.col[beg + m]);
            if (lane == 0) path[s + 1] = nx;
            sb.t = v;
            sb.tb = beg;
            sb.te = beg + d;
            v = nx;
        }
        for (int64_t q = s + 1 + lane; q < L1; q += kWave) path[q] = -1;
        if (lane == 0 && s) atomicAdd(p.steps, (unsigned long long)s);
    }
}

}  // namespace

void launch_walk(const WalkParams& p, int grid, hipStream_t s) {
    if (p.num_walkers <= 0) return;
    const bool flat_n2v = p.bias == kNode2vec && p.w_return == p.w_common && p.w_common == p.w_outward &&
                          p.w_return > 0;
    if (p.bias == kUniform || flat_n2v) {
        int64_t g = (p.num_walkers + kBlock - 1) / kBlock;
        if (g > grid) g = grid;
        hipLaunchKernelGGL(k_walk_uniform, dim3((unsigned)g), dim3(kBlock), 0, s, p);
    } else {
        int64_t g = (p.num_walkers + kWavesPerBlock - 1) / kWavesPerBlock;
        if (g > grid) g = grid;
        hipLaunchKernelGGL(k_walk_wave, dim3((unsigned)g), dim3(kBlock), 0, s, p);
    }
}

}  // namespace csaw
