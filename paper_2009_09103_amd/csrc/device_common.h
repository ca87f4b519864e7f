// device_common.h -- wave64 building blocks for the gfx950 kernels of libcsaw.
//
// Counter-based draws (Philox4x32-10, Salmon et al. SC'11), the exact
// 64-bit range reduction r = floor(u * W / 2^64), and wave-level integer
// scans / reductions / ballots on 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csaw {

constexpr int kWave = 64;
constexpr uint32_t kFallbackRound = 0xFFFFu;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Philox4x32-10 with key (k0, k1) and counter (c0..c3); returns the first two
// output words packed as u = x0 + 2^32 * x1, which is all a draw consumes.
__device__ __forceinline__ uint64_t philox_u64(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                               uint32_t c2, uint32_t c3) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return (uint64_t)c0 | ((uint64_t)c1 << 32);
}

// All four output words of Philox4x32-10 (same rounds as philox_u64).
__device__ __forceinline__ uint4 philox4(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                                         uint32_t c3) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// floor(u * W / 2^64)
__device__ __forceinline__ uint64_t range_reduce(uint64_t u, uint64_t W) { return __umul64hi(u, W); }

struct Key {
    uint32_t k0, k1;
};

__device__ __forceinline__ uint64_t draw(Key key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint64_t W) {
    return range_reduce(philox_u64(key.k0, key.k1, c0, c1, c2, c3), W);
}

// ---------------------------------------------------------------- wave ops
// DPP lane moves (GFX9 encodings): row_shr:n shifts within rows of 16 lanes,
// row_bcast:15 / row_bcast:31 broadcast the last lane of a row (of a row
// pair) into the following row(s). Lanes with no source receive 0. All
// callers run these with every lane of the wave active.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, kCtrl, kRowMask, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), kCtrl, kRowMask, 0xf, false);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Inclusive scan over the 64 lanes (Hillis-Steele inside rows of 16, then
// two row broadcasts).
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x) {
    x += dpp_u64<kDppRowShr1, 0xf>(x);
    x += dpp_u64<kDppRowShr2, 0xf>(x);
    x += dpp_u64<kDppRowShr4, 0xf>(x);
    x += dpp_u64<kDppRowShr8, 0xf>(x);
    x += dpp_u64<kDppRowBcast15, 0xa>(x);
    x += dpp_u64<kDppRowBcast31, 0xc>(x);
    return x;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr1, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr2, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr4, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr8, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowBcast15, 0xa, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowBcast31, 0xc, 0xf, false);
    return x;
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t x, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int lane) {
    const uint32_t lo = readlane_u32((uint32_t)x, lane);
    const uint32_t hi = readlane_u32((uint32_t)(x >> 32), lane);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Sum over the 64 lanes, returned on every lane.
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) { return readlane_u64(wave_incl_scan_u64(x), 63); }

__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) { return (int64_t)wave_sum_u64((uint64_t)x); }

// Width-generic forms for code templated on the prefix type.
__device__ __forceinline__ uint32_t readlane_t(uint32_t x, int lane) { return readlane_u32(x, lane); }
__device__ __forceinline__ uint64_t readlane_t(uint64_t x, int lane) { return readlane_u64(x, lane); }
__device__ __forceinline__ uint32_t wave_incl_scan_t(uint32_t x) { return wave_incl_scan_u32(x); }
__device__ __forceinline__ uint64_t wave_incl_scan_t(uint64_t x) { return wave_incl_scan_u64(x); }

__device__ __forceinline__ int32_t readlane_i32(int32_t x, int lane) {
    return __builtin_amdgcn_readlane(x, lane);
}
__device__ __forceinline__ int64_t readlane_i64(int64_t x, int lane) {
    return (int64_t)readlane_u64((uint64_t)x, lane);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// lanes below the calling lane
__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Make LDS writes of this wave visible to all of its lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave-uniform read through the scalar data cache (constant address space):
// such reads issue back to back and are waited for together, where vector
// loads of one value each, made uniform with readfirstlane, were waited for
// one at a time. Only for data no kernel of the same launch writes.
template <class T>
__device__ __forceinline__ T ld_uniform(const T* p) {
    typedef const __attribute__((address_space(4))) T ConstT;
    return *(ConstT*)p;
}

// v's list [beg, beg + d) of a CSR row-offset view (32-bit words p32 or
// 64-bit p64, one of them set) with both offsets read at once through the
// scalar data cache (v wave-uniform)
template <class Rows>
__device__ __forceinline__ void row_uniform(const Rows& rp, int64_t v, int64_t& beg, int64_t& d) {
    if (rp.p32) {
        const uint32_t a = ld_uniform(rp.p32 + v), b = ld_uniform(rp.p32 + v + 1);
        beg = a;
        d = (int64_t)b - (int64_t)a;
    } else {
        const int64_t a = ld_uniform(rp.p64 + v), b = ld_uniform(rp.p64 + v + 1);
        beg = a;
        d = b - a;
    }
}

// wave-uniform value (forces an SGPR)
__device__ __forceinline__ int32_t uniform_i32(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)((uint64_t)lo | ((uint64_t)hi << 32));
}

}  // namespace csaw
