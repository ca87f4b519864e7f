// mdrw_kernels.hip -- gfx950 kernel of the multi-dimensional random walk
// (frontier sampling, Section II-A; the VertexBias select site of
// fig:api(b)).
//
// One wavefront per instance; its frontier pool lives in LDS (vertex,
// degree, first edge per slot). Lane L owns the slots [L*c, L*c + c),
// c = ceil(P / 64), and keeps their degree total in a register, so a step's
// degree prefix is one 64-lane scan: the owning lane of the draw is the
// number of lanes whose inclusive total is <= r, the slot inside it the
// number of its slots whose running total is <= the remainder. The neighbor
// draw reads one column entry, the new pool vertex's row offsets follow, and
// only the owning lane's total changes. Edges are kept one per lane and
// written 64 steps at a time.
#include "device_common.h"
#include "kernels.h"

namespace csaw {

namespace {

__global__ void __launch_bounds__(kWave) k_mdrw(MdrwParams p) {
    __shared__ int32_t pv[kMaxPool];
    __shared__ uint32_t pd[kMaxPool];
    __shared__ int64_t pb[kMaxPool];
    const int lane = lane_id();
    const Key key{p.k0, p.k1};
    for (int64_t i = blockIdx.x; i < p.num_instances; i += gridDim.x) {
        const int64_t o0 = uniform_i64(p.pool_off[i]);
        const int64_t P = uniform_i64(p.pool_off[i + 1]) - o0;  // <= kMaxPool (checked by the host)
        const uint32_t iid = (uint32_t)(p.instance_base + (uint64_t)i);
        int32_t* src = p.src + i * p.budget;
        int32_t* dst = p.dst + i * p.budget;
        bool bad = false;
        for (int64_t j = lane; j < P; j += kWave) {
            int32_t v = p.pool[o0 + j];
            if (v < 0 || (int64_t)v >= p.g.n) {
                bad = true;
                v = 0;
            }
            const int64_t b = p.g.rowptr[v];
            pv[j] = v;
            pd[j] = (uint32_t)(p.g.rowptr[v + 1] - b);
            pb[j] = b;
        }
        if (ballot(bad)) {  // outputs of the call are unspecified; the host reports the error
            if (lane == 0) *p.bad = 1;
            wave_lds_sync();
            continue;
        }
        wave_lds_sync();
        const int c = (int)((P + kWave - 1) / kWave);
        uint64_t csum = 0;
        for (int q = 0; q < c; ++q) {
            const int64_t j = (int64_t)lane * c + q;
            if (j < P) csum += pd[j];
        }
        int64_t s = 0;
        int32_t bv = -1, bu = -1;  // edge of step s is kept by lane s % 64
        for (; s < p.budget; ++s) {
            const uint64_t incl = wave_incl_scan_u64(csum);
            const uint64_t W = readlane_u64(incl, kWave - 1);
            if (W == 0) break;
            const uint64_t r = draw(key, iid, (uint32_t)s, 0xFFFFFFFFu, 0u, W);
            const int L = __popcll(ballot(incl <= r));  // owning lane of r
            const uint64_t rr = r - readlane_u64(incl - csum, L);
            const int64_t jq = (int64_t)L * c + lane;
            const uint32_t dq = (lane < c && jq < P) ? pd[jq] : 0u;
            const uint64_t iq = wave_incl_scan_u64(dq);
            const int64_t j = (int64_t)L * c + __popcll(ballot(lane < c && iq <= rr));
            const int32_t v = uniform_i32(pv[j]);
            const uint32_t d = (uint32_t)uniform_i32((int32_t)pd[j]);
            const int64_t beg = uniform_i64(pb[j]);
            const uint64_t m = draw(key, iid, (uint32_t)s, (uint32_t)v, 1u, (uint64_t)d);
            const int32_t u = ld_uniform(p.g.col + beg + (int64_t)m);
            int64_t ub, udl;
            row_uniform(p.g.rowptr, u, ub, udl);
            const uint32_t ud = (uint32_t)udl;
            wave_lds_sync();
            if (lane == 0) {
                pv[j] = u;
                pd[j] = ud;
                pb[j] = ub;
            }
            if (lane == L) csum = csum - d + ud;
            wave_lds_sync();
            if (lane == (int)(s & (kWave - 1))) {
                bv = v;
                bu = u;
            }
            if ((s & (kWave - 1)) == kWave - 1) {
                src[s - (kWave - 1) + lane] = bv;
                dst[s - (kWave - 1) + lane] = bu;
            }
        }
        const int64_t s0 = s & ~(int64_t)(kWave - 1);
        if (lane < s - s0) {
            src[s0 + lane] = bv;
            dst[s0 + lane] = bu;
        }
        for (int64_t q = s + lane; q < p.budget; q += kWave) {
            src[q] = -1;
            dst[q] = -1;
        }
        if (lane == 0) {
            if (p.steps) p.steps[i] = s;
            if (s) atomicAdd(p.total, (unsigned long long)s);
        }
        wave_lds_sync();  // the next instance rewrites the pool
    }
}

}  // namespace

void launch_mdrw(const MdrwParams& p, hipStream_t s, LaunchEvents ev) {
    if (p.num_instances <= 0) return;
    const int grid = (int)(p.num_instances < 8192 ? p.num_instances : 8192);
    launch_kernel(k_mdrw, dim3(grid), dim3(kWave), s, ev, p);
}

}  // namespace csaw
