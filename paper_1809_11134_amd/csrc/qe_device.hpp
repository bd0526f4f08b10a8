// Device helpers shared by the libqe kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qe_common.hpp"

namespace qe {

// ---------------------------------------------------------------- Philox4x32-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds
// of two 32x32->64 multiplies with the Weyl key schedule.
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // high and low halves as v_mul_hi_u32 / v_mul_lo_u32 (a single
        // v_mad_u64_u32 per product measured ~3x slower on gfx950)
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ u32x4 draw(uint64_t seed, uint32_t tag, uint32_t gen, uint32_t inst,
                                      uint32_t item) {
    return philox(tag, gen, inst, item, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// floor(w * range / 2^32): a uniform integer in [0, range).
__device__ __forceinline__ uint32_t scale_u32(uint32_t w, uint32_t range) {
    return __umulhi(w, range);
}

// ------------------------------------------------------------------ descriptors
__device__ __forceinline__ int desc_kind(uint32_t d) { return d & 15; }
__device__ __forceinline__ int desc_tgt(uint32_t d) { return (d >> 4) & 15; }
__device__ __forceinline__ int desc_ctl(uint32_t d) { return (d >> 8) & 15; }

// ISING: the circuit carries angles, so the Ising kinds are valid too.
template <bool ISING = false>
__device__ __forceinline__ bool desc_valid(uint32_t d, int n) {
    const int k = d & 15, t = (d >> 4) & 15, c = (d >> 8) & 15;
    if (d >> 12) return false;
    if (k > (ISING ? KIND_ZZ : KIND_T)) return false;
    if (k == KIND_I) return true;
    if (t >= n) return false;
    if (kind_two_wire(k) && (c >= n || c == t)) return false;
    return true;
}

// ------------------------------------------------------------ gate angles
// cos and sin of theta / 2 for an angle stored as a u32 turn fraction
// (theta = 2 pi u / 2^32).  theta / 2 = q pi/2 + pi r / 2^32 with q the
// nearest whole number of quarter turns (0, 1 or 2) and |r| <= 2^30, so the
// reduced argument lies in [-pi/4, pi/4] and is rounded once when r is
// converted; sincospi avoids a rounded multiple of pi.
__device__ __forceinline__ void half_angle(uint32_t u, float* c, float* s) {
    const uint32_t q = (uint32_t)(((uint64_t)u + 0x40000000ull) >> 31);
    const int32_t r = (int32_t)(u - (q << 31));
    float sr, cr;
    sincospif((float)r * 0x1p-32f, &sr, &cr);
    *c = q == 0 ? cr : (q == 1 ? -sr : -cr);
    *s = q == 0 ? sr : (q == 1 ? cr : -sr);
}

__device__ __forceinline__ void half_angle(uint32_t u, double* c, double* s) {
    const uint32_t q = (uint32_t)(((uint64_t)u + 0x40000000ull) >> 31);
    const int32_t r = (int32_t)(u - (q << 31));
    double sr, cr;
    sincospi((double)r * 0x1p-32, &sr, &cr);
    *c = q == 0 ? cr : (q == 1 ? -sr : -cr);
    *s = q == 0 ? sr : (q == 1 ? cr : -sr);
}

// ------------------------------------------------------------- wave reductions
// Sums over the 64 lanes; every lane receives the same value.  All lanes must
// be active.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// FP32 version without LDS round trips: DPP within rows of 16 lanes (lane
// l ^ 1, l ^ 2, the mirror inside 8 lanes, the mirror inside 16), then the
// row swaps of v_permlane16_swap / v_permlane32_swap.  Each step adds the
// same two partial sums on both partner lanes, so the result is identical
// everywhere.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v),
                                                        false, false);
        v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v),
                                                        false, false);
        v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    return v;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

}  // namespace qe
