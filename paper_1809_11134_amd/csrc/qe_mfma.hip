// Fused dense gate blocks on MFMA (n = 5, 6).
//
// Consecutive gates whose wires fit in a window of 4 wires are fused into a
// 16 x 16 complex block B (built by applying them to the identity), and B is
// applied to U T^dagger as one dense product: for every setting b of the
// wires outside the window and every column j, the 16 entries of column j on
// the window rows are multiplied by B.  As a real GEMM the block is
// [[Re B, -Im B], [Im B, Re B]] (32 x 32) times the 32 x (2^(n-4) N) stack of
// real and imaginary parts, done with v_mfma_f32_32x32x16_{bf16,f16}: every
// operand x is split as x = hi + lo (hi = x rounded to 16 bits, lo = the
// rounded remainder; fp16 lo scaled by 2^11 to stay normal) and
// hi*hi + hi*lo + lo*hi is accumulated in FP32.  Optionally every column of
// U T^dagger is rescaled to unit norm after each block (the columns of a
// unitary have unit norm; the rescaling removes the drift of the rounding).
//
// A group with fewer than `min_block` non-identity gates is not worth a
// block (building B and the three products cost more than a few row-pair
// updates): its gates are applied to U T^dagger one by one in FP32, as the
// LDS-staged path does.  min_block = 1 fuses every group; the autotuner
// chooses it per width and length class.
//
// Layout: U T^dagger lives in LDS as in the LDS-staged FP32 path, and the
// W wavefronts of a circuit own 16 columns each, so no barrier is needed
// between blocks; each wavefront builds its own copy of B in a 2 KB LDS
// scratch.  GEMM columns are ordered (j, b) so that a wavefront's MFMA tiles
// cover exactly its own columns.
#include "../../include/qe.h"
#include "qe_eval_core.hpp"
#include "qe_internal.hpp"

namespace qe {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <bool FP16>
struct Mma;

template <>
struct Mma<false> {
    using E = __bf16;
    using V = bf16x8;
    static constexpr float LO = 1.0f;
    __device__ static __forceinline__ void split(float x, E& h, E& l) {
        h = (E)x;
        l = (E)(x - (float)h);
    }
    __device__ static __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

template <>
struct Mma<true> {
    using E = _Float16;
    using V = f16x8;
    static constexpr float LO = 2048.0f;
    __device__ static __forceinline__ void split(float x, E& h, E& l) {
        h = (E)x;
        l = (E)((x - (float)h) * 2048.0f);
    }
    __device__ static __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// Deposits the 4 bits of a (bit 3 = window wire 0) at the row-bit positions
// of the window wires wq[0..3] (row bit of wire w is n-1-w).
// (wq: 4 bits per window wire, wire q in bits 4q..4q+3.)
__device__ __forceinline__ int deposit4(int a, uint32_t wq, int n) {
    int i = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) i |= ((a >> (3 - q)) & 1) << (n - 1 - (int)((wq >> (4 * q)) & 15));
    return i;
}

// Applies the group's gates (lanes first..first+cnt-1 of the descriptor
// chunk dv, wires remapped to the window) to the identity in the
// wavefront's 16 x 16 scratch B.
__device__ __forceinline__ void build_block(float2* B, uint32_t dv, int first, int cnt,
                                            uint32_t wpos) {
    const int lane = (int)lane_id();
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const int e = lane + 64 * h;
        B[e] = make_float2((e >> 4) == (e & 15) ? 1.0f : 0.0f, 0.0f);
    }
    wave_lds_fence();
    const float r = 0.70710678118654752f;
    for (int g = first; g < first + cnt; ++g) {
        const uint32_t d = __builtin_amdgcn_readlane(dv, g);
        const int kind = d & 15;
        if (kind == KIND_I) continue;
        const int tpos = 3 - (int)((wpos >> (4 * ((d >> 4) & 15))) & 15);
        const int tb = 1 << tpos;
        const int cb = kind_controlled(kind) ? 1 << (3 - (int)((wpos >> (4 * ((d >> 8) & 15))) & 15)) : 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = lane + 64 * h;          // 8 row pairs x 16 columns
            const int pr = p >> 4, j = p & 15;
            const int i0 = ins0(pr, tpos), i1 = i0 | tb;
            if (cb && !(i0 & cb)) continue;
            const float2 a = B[i0 * 16 + j], b = B[i1 * 16 + j];
            float2 x = a, y = b;
            if (kind == KIND_NOT || kind == KIND_CNOT) {
                x = b; y = a;
            } else if (kind == KIND_CV || kind == KIND_CVDG) {
                const float p_ = a.x + b.x, q = a.y + b.y, u = a.x - b.x, v = a.y - b.y;
                const float2 s0 = make_float2(0.5f * (p_ - v), 0.5f * (q + u));
                const float2 s1 = make_float2(0.5f * (p_ + v), 0.5f * (q - u));
                x = kind == KIND_CV ? s0 : s1;
                y = kind == KIND_CV ? s1 : s0;
            } else if (kind == KIND_H) {
                x = make_float2((a.x + b.x) * r, (a.y + b.y) * r);
                y = make_float2((a.x - b.x) * r, (a.y - b.y) * r);
            } else {
                y = make_float2((b.x - b.y) * r, (b.x + b.y) * r);
            }
            B[i0 * 16 + j] = x;
            B[i1 * 16 + j] = y;
        }
        wave_lds_fence();
    }
}

// One gate (descriptor d, wires of the circuit) applied to the wavefront's
// 16 columns of U T^dagger: lane l takes column jbase + l mod 16 and the row
// pairs whose pair index is l div 16 modulo 4.
template <int NQ>
__device__ __forceinline__ void gate_on_columns(float2* M, uint32_t d, int jbase) {
    constexpr int N = 1 << NQ, RG = 4;
    const int lane = (int)lane_id();
    const int j = jbase + (lane & 15), rg = lane >> 4;
    const int kind = d & 15;
    const int tpos = NQ - 1 - (int)((d >> 4) & 15);
    const int tb = 1 << tpos;
    const int cb = kind_controlled(kind) ? 1 << (NQ - 1 - (int)((d >> 8) & 15)) : 0;
    const float r = 0.70710678118654752f;
#pragma unroll
    for (int m = 0; m < N / 2 / RG; ++m) {
        const int i0 = ins0(rg + RG * m, tpos), i1 = i0 | tb;
        if (cb && !(i0 & cb)) continue;
        const float2 a = M[i0 * N + j], b = M[i1 * N + j];
        float2 x = a, y = b;
        if (kind == KIND_NOT || kind == KIND_CNOT) {
            x = b; y = a;
        } else if (kind == KIND_CV || kind == KIND_CVDG) {
            const float p_ = a.x + b.x, q = a.y + b.y, u = a.x - b.x, v = a.y - b.y;
            const float2 s0 = make_float2(0.5f * (p_ - v), 0.5f * (q + u));
            const float2 s1 = make_float2(0.5f * (p_ + v), 0.5f * (q - u));
            x = kind == KIND_CV ? s0 : s1;
            y = kind == KIND_CV ? s1 : s0;
        } else if (kind == KIND_H) {
            x = make_float2((a.x + b.x) * r, (a.y + b.y) * r);
            y = make_float2((a.x - b.x) * r, (a.y - b.y) * r);
        } else {
            y = make_float2((b.x - b.y) * r, (b.x + b.y) * r);
        }
        M[i0 * N + j] = x;
        M[i1 * N + j] = y;
    }
}

template <int NQ, bool FP16>
__device__ __forceinline__ void apply_block(float2* M, const float2* B, uint32_t wq,
                                            uint32_t ow, int jbase, bool renorm) {
    using T = Mma<FP16>;
    constexpr int N = 1 << NQ, NB = 1 << (NQ - 4);
    constexpr int TILES = 16 * NB / 32;      // MFMA column tiles of this wave's 16 columns
    const int lane = (int)lane_id();
    const int half = lane >> 5, ln = lane & 31;
    // A operand: real embedding of B, rows m = ln, k = half*8 + q (K step 0:
    // the real-part columns, K step 1: the imaginary-part columns)
    typename T::V A0h, A0l, A1h, A1l;
    {
        const int m = ln & 15;
        const bool top = ln < 16;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float2 v = B[m * 16 + half * 8 + q];
            const float s0 = top ? v.x : v.y;      // [Re B | -Im B] over [Im B | Re B]
            const float s1 = top ? -v.y : v.x;
            typename T::E h, l;
            T::split(s0, h, l); A0h[q] = h; A0l[q] = l;
            T::split(s1, h, l); A1h[q] = h; A1l[q] = l;
        }
    }
    // window part of the row index of this lane's K rows (a' = half*8 + q)
    // and of its output rows (a = (r/4)*8 + half*4 + r%4)
    int rin[8], rout[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        rin[q] = deposit4(half * 8 + q, wq, NQ);
        rout[q] = deposit4((q >> 2) * 8 + half * 4 + (q & 3), wq, NQ);
    }
#pragma unroll
    for (int t = 0; t < TILES; ++t) {
        const int col = t * 32 + ln;           // GEMM column (j, b) of this wave
        const int j = jbase + col / NB, b = col % NB;
        int brow = 0;
#pragma unroll
        for (int r = 0; r < NQ - 4; ++r)
            brow |= ((b >> (NQ - 5 - r)) & 1) << (NQ - 1 - (int)((ow >> (4 * r)) & 15));
        typename T::V X0h, X0l, X1h, X1l;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float2 v = M[(brow | rin[q]) * N + j];
            typename T::E h, l;
            T::split(v.x, h, l); X0h[q] = h; X0l[q] = l;
            T::split(v.y, h, l); X1h[q] = h; X1l[q] = l;
        }
        f32x16 c = {}, cx = {};
        c = T::mma(A0h, X0h, c);
        c = T::mma(A1h, X1h, c);
        cx = T::mma(A0h, X0l, cx);
        cx = T::mma(A1h, X1l, cx);
        cx = T::mma(A0l, X0h, cx);
        cx = T::mma(A1l, X1h, cx);
        float re[8], im[8];
        float nrm = 0.0f;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            re[r] = c[r] + cx[r] * (1.0f / T::LO);
            im[r] = c[r + 8] + cx[r + 8] * (1.0f / T::LO);
            nrm += re[r] * re[r] + im[r] * im[r];
        }
        if (renorm) {
            // lanes sharing column j: the NB values of b and both halves
#pragma unroll
            for (int m = 1; m < NB; m <<= 1) nrm += __shfl_xor(nrm, m, 64);
            nrm += __shfl_xor(nrm, 32, 64);
            const float sc = nrm > 0.0f ? 1.0f / sqrtf(nrm) : 1.0f;
#pragma unroll
            for (int r = 0; r < 8; ++r) { re[r] *= sc; im[r] *= sc; }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) M[(brow | rout[r]) * N + j] = make_float2(re[r], im[r]);
    }
}

template <int NQ, bool FP16>
__global__ __launch_bounds__(64 * (1 << (NQ - 4))) void mfma_kernel(BatchArgs a, float* __restrict__ f,
                                                                   float* __restrict__ g,
                                                                   float* __restrict__ delta,
                                                                   int renorm, int min_block) {
    constexpr int N = 1 << NQ, W = N / 16, CW = 16, RG = 64 / CW;
    __shared__ float2 M[N * N];
    __shared__ float2 Bs[W][256];
    __shared__ float red[W][3];
    const int b = blockIdx.x;
    const int lane = (int)lane_id(), wave = (int)(threadIdx.x >> 6);
    Item it = resolve_item(a, b, true);
    if (it.err == 0 && it.n != NQ) it.err = QE_DEVERR_WIDTH;
    bool ok = it.err == 0;
    const int jl = lane % CW, rg = lane / CW, j = wave * CW + jl;
    if (ok) {
        const float2* T2 = reinterpret_cast<const float2*>(a.targets) + it.toff;
#pragma unroll
        for (int m = 0; m < N / RG; ++m) {
            const int r = m * RG + rg;
            float2 v = T2[(size_t)j * N + r];
            v.y = -v.y;
            M[r * N + j] = v;
        }
        wave_lds_fence();
        // greedy grouping of consecutive gates into windows of <= 4 wires
        const int L = it.L;
        const uint16_t* gp = it.g;
        uint32_t gmask = 0, dv = 0;
        int gstart = 0, gcnt = 0, gnon = 0;
        auto flush = [&]() {
            if (gcnt == 0) return;
            if (gnon < min_block) {
                // too few gates for a block: one by one, in FP32
                for (int k = gstart; k < gstart + gcnt; ++k) {
                    const uint32_t d = __builtin_amdgcn_readlane(dv, k);
                    if ((d & 15) == KIND_I) continue;
                    gate_on_columns<NQ>(M, d, wave * CW);
                    wave_lds_fence();
                }
                gmask = 0;
                gcnt = 0;
                gnon = 0;
                return;
            }
            // window = the group's wires padded with the lowest unused ones;
            // packed 4 bits per entry: wq (window wire of position q), wpos
            // (position of each wire), ow (the other wires, ascending)
            uint32_t m = gmask;
            for (int w = 0; w < NQ && __builtin_popcount(m) < 4; ++w) m |= 1u << w;
            uint32_t wq = 0, wpos = 0, ow = 0;
            int q = 0, o = 0;
            for (int w = 0; w < NQ; ++w) {
                if (m & (1u << w)) { wpos |= (uint32_t)q << (4 * w); wq |= (uint32_t)w << (4 * q); ++q; }
                else { ow |= (uint32_t)w << (4 * o); ++o; }
            }
            build_block(Bs[wave], dv, gstart, gcnt, wpos);
            apply_block<NQ, FP16>(M, Bs[wave], wq, ow, wave * CW, renorm != 0);
            wave_lds_fence();
            gmask = 0;
            gcnt = 0;
            gnon = 0;
        };
        // groups never straddle a chunk of 64 descriptors (positions within
        // the chunk index the register dv)
        for (int ch = 0; ch * 64 < L && ok; ++ch) {
            const int p = ch * 64 + lane;
            dv = p < L ? (uint32_t)gp[p] : 0u;
            const int cnt = min(64, L - ch * 64);
            if (__ballot((lane < cnt) && !desc_valid(dv, NQ))) { ok = false; break; }
            for (int k = 0; k < cnt; ++k) {
                const uint32_t d = __builtin_amdgcn_readlane(dv, k);
                const int kind = d & 15;
                if (kind == KIND_I) continue;
                uint32_t wm = 1u << ((d >> 4) & 15);
                if (kind_controlled(kind)) wm |= 1u << ((d >> 8) & 15);
                if (gcnt > 0 && __builtin_popcount(gmask | wm) > 4) flush();
                if (gcnt == 0) gstart = k;
                // a group is a contiguous run of the stream (identities inside are kept)
                gcnt = k - gstart + 1;
                gmask |= wm;
                ++gnon;
            }
            flush();
        }
        if (!ok) it.err = QE_DEVERR_DESC;
    }
    // fitness (as the LDS-staged FP32 path)
    float off = 0.0f;
    float2 dg = make_float2(0.0f, 0.0f);
    if (ok) {
#pragma unroll
        for (int m = 0; m < N / RG; ++m) {
            const int r = m * RG + rg;
            const float2 v = M[r * N + j];
            off += (r == j) ? 0.0f : v.x * v.x + v.y * v.y;
        }
        if (lane < CW) dg = M[j * N + j];
    }
    const float offw = wave_sum(off), trw = wave_sum(dg.x), tiw = wave_sum(dg.y);
    if (lane == 0) { red[wave][0] = offw; red[wave][1] = trw; red[wave][2] = tiw; }
    __syncthreads();
    float offs = 0.0f, tr = 0.0f, ti = 0.0f;
#pragma unroll
    for (int w = 0; w < W; ++w) { offs += red[w][0]; tr += red[w][1]; ti += red[w][2]; }
    const float am = sqrtf(tr * tr + ti * ti);
    float er = 1.0f, ei = 0.0f;
    if (am > 0.0f) { er = tr / am; ei = ti / am; }
    float dl = 0.0f;
    if (lane < CW) { const float xr = dg.x - er, xi = dg.y - ei; dl = xr * xr + xi * xi; }
    const float dw = wave_sum(dl);
    __syncthreads();
    if (lane == 0) red[wave][0] = dw;
    __syncthreads();
    if (threadIdx.x == 0) {
        float D = 0.0f;
#pragma unroll
        for (int w = 0; w < W; ++w) D += red[w][0];
        float dlt = 0.5f * (offs + D);
        const float q = fminf(fmaxf(dlt / (float)N, 0.0f), 1.0f);
        float fv = 1.0f - sqrtf(q), gv = am / (float)N;
        if (a.mode == QE_FIT_PHASE_INSENSITIVE) fitness_pi(offs, N, &fv, &gv, &dlt);
        const float nan = __builtin_nanf("");
        if (ok && !(fv == fv)) it.err = QE_DEVERR_NUMERIC;
        f[b] = ok ? fv : nan;
        if (g) g[b] = ok ? gv : nan;
        if (delta) delta[b] = ok ? dlt : nan;
        if (it.err) atomicOr(a.err, it.err);
    }
}

hipError_t launch_eval_mfma(const BatchArgs& a, bool fp16, bool renorm, float* f, float* g,
                            float* delta, hipStream_t s) {
    if (a.B == 0) return hipSuccess;
    const int rn = renorm ? 1 : 0;
    const int mb = mfma_min_block(a.uniform_n, a.uniform_L > 0 ? a.uniform_L : 32);
    if (a.uniform_n == 5) {
        if (fp16) mfma_kernel<5, true><<<a.B, 128, 0, s>>>(a, f, g, delta, rn, mb);
        else mfma_kernel<5, false><<<a.B, 128, 0, s>>>(a, f, g, delta, rn, mb);
    } else if (a.uniform_n == 6) {
        if (fp16) mfma_kernel<6, true><<<a.B, 256, 0, s>>>(a, f, g, delta, rn, mb);
        else mfma_kernel<6, false><<<a.B, 256, 0, s>>>(a, f, g, delta, rn, mb);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qe
