// Per-circuit evaluation cores (one wavefront per circuit), gfx950.
//
// The hot path builds M = U T^dagger gate by gate starting from M_0 = T^dagger:
// a gate G on wires (c, t) left-multiplies M, i.e. it mixes pairs of rows
// (i, i ^ target bit) whose control bit is set.  tr(M_L) = tr(T^dagger U)
// gives Eq. 11 of Sec. IV-E; the residual ||M_L - e^{i arg tr} I||_F^2 / 2
// gives the same radicand without cancellation.
//
// Register layout (n = 4, 5, 6): the N x N complex matrix (N = 2^n) is spread
// over the 64 lanes of a wavefront and E = N^2 / 64 registers per lane.  The
// column index j occupies lane bits 0..n-1 and never moves (gates act on rows
// only).  The n row bits ("slots") live either in register-index bits
// 0..EB-1 (EB = 2n - 6) or in lane bits n..5.  A wave-uniform map records
// which wire sits in which slot.  Before a gate the target wire is moved to
// register bit 0 and a register-resident control to register bit EB-1, by
// exchanging register bits (register renames) or a lane bit with a register
// bit (v_permlane16/32_swap); a lane-resident control becomes an exec
// predicate.  Every gate body is then one of a handful of fully unrolled
// register loops, and no shuffle or LDS traffic is needed for the arithmetic.
//
// LDS-staged layout (n = 4..6, the tuned default; run_lds_path): M lives in
// LDS, W wavefronts split its columns, each lane updates the row pairs of one
// column per pass, and the gate constants come from a per-chunk gate program.
// One entry per lane (n <= 3; run_small_path): lane l holds M[l / N][l % N].
//
// Gate sources.  A path reads the circuit through a callable src(chunk) that
// returns this lane's gate of the chunk: a uint32 descriptor for the
// discrete libraries, or a uint2 {descriptor, angle} when the circuit may
// hold Ising gates (kinds 7-10, angle a u32 turn fraction).  The angled
// form compiles the Ising kinds in; the register-resident path takes the
// discrete form only.
#pragma once
#include <type_traits>

#include "../../include/qe.h"
#include "qe_device.hpp"
#include "qe_internal.hpp"

namespace qe {

// ------------------------------------------------------------ batch items
struct Item {
    int n, L;
    const uint16_t* g;
    const uint32_t* ang;   // the circuit's angles, or null
    int64_t toff;
    uint32_t err;
};

// Resolves circuit b of a batch (wave-uniform) and checks it against the
// buffer bounds; err != 0 means the circuit must not be evaluated.
__device__ __forceinline__ Item resolve_item(const BatchArgs& a, int b, bool need_target) {
    Item it;
    it.err = 0;
    it.n = a.uniform_n > 0 ? a.uniform_n : (int)a.nq[b];
    it.L = 0;
    it.g = a.gates;
    it.ang = a.angles;
    it.toff = 0;
    if (it.n < 1 || it.n > MAX_QUBITS) { it.err = QE_DEVERR_WIDTH; return it; }
    int64_t start, end;
    if (a.uniform_L > 0) {
        start = (int64_t)b * a.uniform_L;
        end = start + a.uniform_L;
    } else {
        start = a.goff[b];
        end = a.goff[b + 1];
    }
    if (start < 0 || end < start || end > a.num_gates) { it.err = QE_DEVERR_RANGE; return it; }
    it.L = (int)(end - start);
    it.g = a.gates + start;
    it.ang = a.angles ? a.angles + start : nullptr;
    if (!need_target) return it;
    const int64_t NN = (int64_t)1 << (2 * it.n);
    it.toff = a.tstride >= 0 ? (int64_t)b * a.tstride : a.toff[b];
    if (it.toff < 0 || it.toff + NN > a.num_telems) { it.err = QE_DEVERR_RANGE; return it; }
    return it;
}

__device__ __forceinline__ float bits_f(uint32_t u) { return __uint_as_float(u); }

// ---------------------------------------------------------- gate sources
template <typename GateSrc>
constexpr bool src_angled() {
    return std::is_same<std::decay_t<decltype(std::declval<GateSrc&>()(0))>, uint2>::value;
}
__device__ __forceinline__ uint32_t desc_of(uint32_t v) { return v; }
__device__ __forceinline__ uint32_t desc_of(uint2 v) { return v.x; }
__device__ __forceinline__ uint32_t angle_of(uint32_t) { return 0u; }
__device__ __forceinline__ uint32_t angle_of(uint2 v) { return v.y; }

// Ising gate on a pair of rows (a: target bit 0, b: target bit 1) with
// c, s = cos, sin of theta / 2 (Eqs. 3-5): R_x mixes with -i s, R_y with
// -+ s, R_z multiplies a by e^{-i theta/2} and b by e^{i theta/2}.
__device__ __forceinline__ float2 phase_minus(float2 x, float c, float s) {   // x (c - i s)
    return make_float2(c * x.x + s * x.y, c * x.y - s * x.x);
}
__device__ __forceinline__ float2 phase_plus(float2 x, float c, float s) {    // x (c + i s)
    return make_float2(c * x.x - s * x.y, c * x.y + s * x.x);
}
__device__ __forceinline__ uint32_t f_bits(float f) { return __float_as_uint(f); }

// ----------------------------------------------------------- lane-bit swaps
// Exchange lane bit 5 (LB = 5) or lane bit 4 (LB = 4) of the elements of
// registers a (register bit 0) and b (register bit 1): after the call a holds
// in its upper half-lanes what b held in its lower ones and vice versa.
template <int LB>
__device__ __forceinline__ void lane_swap(float& a, float& b) {
    if constexpr (LB == 5) {
        auto r = __builtin_amdgcn_permlane32_swap(f_bits(a), f_bits(b), false, false);
        a = bits_f(r[0]);
        b = bits_f(r[1]);
    } else {
        static_assert(LB == 4, "lane bit");
        auto r = __builtin_amdgcn_permlane16_swap(f_bits(a), f_bits(b), false, false);
        a = bits_f(r[0]);
        b = bits_f(r[1]);
    }
}

// ------------------------------------------------------------ register swaps
// In-place exchange of two VGPRs.  Written as v_swap_b32 so that the values
// stay in the registers the allocator gave the two variables: a plain C++
// swap becomes a pair of renamed values that must be copied back at every
// control-flow merge of the gate dispatch.
__device__ __forceinline__ void vswap(float& a, float& b) {
    asm volatile("v_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}

// Exchange register bits A < B: element k with bit A set and bit B clear
// trades places with k ^ (1<<A) ^ (1<<B).
template <int E, int A, int B>
__device__ __forceinline__ void swap_reg_bits(float* re, float* im) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
        if (((k >> A) & 1) == 1 && ((k >> B) & 1) == 0) {
            const int k2 = k ^ (1 << A) ^ (1 << B);
            vswap(re[k], re[k2]);
            vswap(im[k], im[k2]);
        }
    }
}

// Exchange register bit R with lane bit LB.
template <int E, int R, int LB>
__device__ __forceinline__ void swap_lane_reg(float* re, float* im) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
        if (((k >> R) & 1) == 0) {
            const int k2 = k | (1 << R);
            lane_swap<LB>(re[k], re[k2]);
            lane_swap<LB>(im[k], im[k2]);
        }
    }
}

template <int E, int EB>
__device__ __forceinline__ void swap_reg_rt(int a, int b, float* re, float* im) {
    // a < b < EB (wave-uniform)
#define QE_SW(A, B)                                                  \
    case (A)*8 + (B):                                                \
        if constexpr ((B) < EB) swap_reg_bits<E, A, B>(re, im);      \
        break;
    switch (a * 8 + b) {
        QE_SW(0, 1) QE_SW(0, 2) QE_SW(0, 3) QE_SW(0, 4) QE_SW(0, 5)
        QE_SW(1, 2) QE_SW(1, 3) QE_SW(1, 4) QE_SW(1, 5)
        QE_SW(2, 3) QE_SW(2, 4) QE_SW(2, 5)
        QE_SW(3, 4) QE_SW(3, 5)
        QE_SW(4, 5)
        default: break;
    }
#undef QE_SW
}

template <int E, int EB>
__device__ __forceinline__ void swap_lane_reg_rt(int r, int lb, float* re, float* im) {
#define QE_LR(R)                                                                   \
    case R:                                                                        \
        if constexpr ((R) < EB) {                                                  \
            if (lb == 5) swap_lane_reg<E, R, 5>(re, im);                           \
            else swap_lane_reg<E, R, 4>(re, im);                                   \
        }                                                                          \
        break;
    switch (r) {
        QE_LR(0) QE_LR(1) QE_LR(2) QE_LR(3) QE_LR(4) QE_LR(5)
        default: break;
    }
#undef QE_LR
}

// ------------------------------------------------------------------ slot map
// Wave-uniform map between wires and slots, 4 bits per entry.
struct SlotMap {
    uint32_t w2s, s2w;
    __device__ __forceinline__ int slot(int w) const { return (w2s >> (4 * w)) & 15; }
    __device__ __forceinline__ int wire(int s) const { return (s2w >> (4 * s)) & 15; }
    __device__ __forceinline__ void exchange(int a, int b) {
        const int wa = wire(a), wb = wire(b);
        s2w = (s2w & ~(15u << (4 * a)) & ~(15u << (4 * b))) | ((uint32_t)wb << (4 * a)) |
              ((uint32_t)wa << (4 * b));
        w2s = (w2s & ~(15u << (4 * wa)) & ~(15u << (4 * wb))) | ((uint32_t)b << (4 * wa)) |
              ((uint32_t)a << (4 * wb));
    }
};

// Exchange the contents of slots a != b (register bit < EB or lane bit).
template <int NQ, int E, int EB>
__device__ __forceinline__ void swap_slots(int a, int b, float* re, float* im, SlotMap& map) {
    if (a > b) { const int t = a; a = b; b = t; }
    if constexpr (EB == NQ) {   // every slot is a register bit
        swap_reg_rt<E, EB>(a, b, re, im);
    } else if (b < EB) {
        swap_reg_rt<E, EB>(a, b, re, im);
    } else if (a < EB) {
        swap_lane_reg_rt<E, EB>(a, NQ + b - EB, re, im);
    } else {
        // both in lanes (n = 4): route through register bit 0
        swap_lane_reg_rt<E, EB>(0, NQ + a - EB, re, im);
        swap_lane_reg_rt<E, EB>(0, NQ + b - EB, re, im);
        swap_lane_reg_rt<E, EB>(0, NQ + a - EB, re, im);
    }
    map.exchange(a, b);
}

// ---------------------------------------------------------------- gate bodies
// Target at register bit 0.  CTL: 0 = uncontrolled, 1 = control at register
// bit EB-1 (only the upper half of the registers is transformed).
template <int E, int CTL>
__device__ __forceinline__ void body_x(float* re, float* im) {
#pragma unroll
    for (int k = (CTL ? E / 2 : 0); k < E; k += 2) {
        vswap(re[k], re[k + 1]);
        vswap(im[k], im[k + 1]);
    }
}

// V = (1/2)[[1+i, 1-i], [1-i, 1+i]]:  a' = (s + i d)/2, b' = (s - i d)/2 with
// s = a + b, d = a - b.  V^dagger swaps the two outputs.
template <int E, int CTL, bool DAG>
__device__ __forceinline__ void body_v(float* re, float* im) {
#pragma unroll
    for (int k = (CTL ? E / 2 : 0); k < E; k += 2) {
        const float p = re[k] + re[k + 1], q = im[k] + im[k + 1];
        const float u = re[k] - re[k + 1], v = im[k] - im[k + 1];
        const float xr = 0.5f * (p - v), xi = 0.5f * (q + u);
        const float yr = 0.5f * (p + v), yi = 0.5f * (q - u);
        if (DAG) { re[k] = yr; im[k] = yi; re[k + 1] = xr; im[k + 1] = xi; }
        else     { re[k] = xr; im[k] = xi; re[k + 1] = yr; im[k + 1] = yi; }
    }
}

template <int E>
__device__ __forceinline__ void body_h(float* re, float* im) {
    const float r = 0.70710678118654752f;
#pragma unroll
    for (int k = 0; k < E; k += 2) {
        const float ar = re[k], ai = im[k], br = re[k + 1], bi = im[k + 1];
        re[k] = (ar + br) * r; im[k] = (ai + bi) * r;
        re[k + 1] = (ar - br) * r; im[k + 1] = (ai - bi) * r;
    }
}

template <int E>
__device__ __forceinline__ void body_t(float* re, float* im) {
    const float r = 0.70710678118654752f;   // e^{i pi/4} = (1 + i)/sqrt(2)
#pragma unroll
    for (int k = 1; k < E; k += 2) {
        const float br = re[k], bi = im[k];
        re[k] = (br - bi) * r;
        im[k] = (br + bi) * r;
    }
}

// --------------------------------------------------------- fitness reduction
struct FitOut {
    float f, g, delta;
};

// Phase-insensitive fitness (QE_FIT_PHASE_INSENSITIVE) from the energy of M
// off its diagonal: for unitary M, 1 - sum_i |M_ii|^2 / N = off / N, so the
// radicand needs no subtraction.
template <typename Real>
__device__ __forceinline__ void fitness_pi(Real offs, int N, Real* f, Real* g, Real* delta) {
    const Real r = offs / (Real)N;
    const Real q = r < (Real)0 ? (Real)0 : (r > (Real)1 ? (Real)1 : r);
    *f = (Real)1 - sqrt(q);
    *g = (Real)1 - r;
    *delta = offs;
}

// Reduction of M (held as per-lane partial sums: off-diagonal |m|^2 and the
// lane's diagonal element, if any) into Eq. 11, or (mode) the
// phase-insensitive fitness.
__device__ __forceinline__ FitOut finish_fitness(float off, float dre, float dim, bool hasd,
                                                 int N, int mode = QE_FIT_EQ11) {
    const float offs = wave_sum(off);
    if (mode == QE_FIT_PHASE_INSENSITIVE) {
        FitOut o;
        fitness_pi(offs, N, &o.f, &o.g, &o.delta);
        if (!(o.f == o.f)) o.f = __builtin_nanf("");
        return o;
    }
    const float tre = wave_sum(dre), tim = wave_sum(dim);
    const float a = sqrtf(tre * tre + tim * tim);
    float er = 1.0f, ei = 0.0f;
    if (a > 0.0f) { er = tre / a; ei = tim / a; }
    float dl = 0.0f;
    if (hasd) {
        const float xr = dre - er, xi = dim - ei;
        dl = xr * xr + xi * xi;
    }
    const float D = wave_sum(dl);
    const float delta = 0.5f * (offs + D);
    float q = delta / (float)N;
    q = fminf(fmaxf(q, 0.0f), 1.0f);
    FitOut o;
    o.f = 1.0f - sqrtf(q);
    o.g = a / (float)N;
    o.delta = delta;
    if (!(o.f == o.f) || !(delta == delta)) o.f = __builtin_nanf("");
    return o;
}

// -------------------------------------------------------- register-path core
// GateSrc: callable chunk(c) -> this lane's descriptor for position
// c*64 + lane (0 beyond the circuit), evaluated by all lanes.
// Returns false if a descriptor was invalid (the result is then garbage).
template <int NQ, bool IDENT, typename GateSrc>
__device__ __forceinline__ bool run_register_path(const float* __restrict__ T, int L,
                                                  GateSrc&& src, float* U_out, FitOut* fit,
                                                  int mode = QE_FIT_EQ11) {
    constexpr int N = 1 << NQ;
    constexpr int E = N * N / 64;
    constexpr int EB = 2 * NQ - 6;
    const int lane = (int)lane_id();
    const int j = lane & (N - 1);
    const int lr = lane >> NQ;
    const uint32_t dv0 = L > 0 ? src(0) : 0u;   // before the target: latencies overlap
    float re[E], im[E];
    if (IDENT) {
#pragma unroll
        for (int k = 0; k < E; ++k) {
            re[k] = ((k | (lr << EB)) == j) ? 1.0f : 0.0f;
            im[k] = 0.0f;
        }
    } else {
        // M_0 = T^dagger: element (i, j) = conj(T[j][i]); this lane's rows are
        // i = lr*E + k, contiguous in row j of T.
        const float2* src2 = reinterpret_cast<const float2*>(T) + (size_t)j * N + (size_t)lr * E;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const float2 v = src2[k];
            re[k] = v.x;
            im[k] = -v.y;
        }
    }
    // canonical map: wire w in slot n-1-w
    SlotMap map;
    map.w2s = 0; map.s2w = 0;
#pragma unroll
    for (int w = 0; w < NQ; ++w) {
        map.w2s |= (uint32_t)(NQ - 1 - w) << (4 * w);
        map.s2w |= (uint32_t)w << (4 * (NQ - 1 - w));
    }
    bool ok = true;
    const int chunks = (L + 63) >> 6;
    for (int ch = 0; ch < chunks; ++ch) {
        const uint32_t dv = ch == 0 ? dv0 : src(ch);
        const int cnt = min(64, L - ch * 64);
        const bool bad = (lane < cnt) && !desc_valid(dv, NQ);
        if (__ballot(bad)) { ok = false; break; }
        for (int g = 0; g < cnt; ++g) {
            const uint32_t d = __builtin_amdgcn_readlane(dv, g);
            const int kind = d & 15;
            if (kind == KIND_I) continue;
            const int t = (d >> 4) & 15;
            const int st = map.slot(t);
            if (st != 0) swap_slots<NQ, E, EB>(st, 0, re, im, map);
            if (kind_controlled(kind)) {
                const int c = (d >> 8) & 15;
                const int sc = map.slot(c);
                if (sc < EB) {
                    if (sc != EB - 1) swap_slots<NQ, E, EB>(sc, EB - 1, re, im, map);
                    if (kind == KIND_CNOT) body_x<E, 1>(re, im);
                    else if (kind == KIND_CV) body_v<E, 1, false>(re, im);
                    else body_v<E, 1, true>(re, im);
                } else {
                    const bool on = (lane >> (NQ + sc - EB)) & 1;
                    if (on) {
                        if (kind == KIND_CNOT) body_x<E, 0>(re, im);
                        else if (kind == KIND_CV) body_v<E, 0, false>(re, im);
                        else body_v<E, 0, true>(re, im);
                    }
                }
            } else if (kind == KIND_NOT) {
                body_x<E, 0>(re, im);
            } else if (kind == KIND_H) {
                body_h<E>(re, im);
            } else {
                body_t<E>(re, im);
            }
        }
    }
    // back to the canonical map (wire w in slot n-1-w)
#pragma unroll
    for (int w = 0; w < NQ; ++w) {
        const int want = NQ - 1 - w;
        const int s = map.slot(w);
        if (s != want) swap_slots<NQ, E, EB>(s, want, re, im, map);
    }
    if (U_out) {
        float2* dst = reinterpret_cast<float2*>(U_out);
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int i = k | (lr << EB);
            dst[(size_t)i * N + j] = make_float2(re[k], im[k]);
        }
    }
    if (fit) {
        const int key = ((j >> EB) == lr) ? (j & (E - 1)) : -1;
        float off = 0.0f, dre = 0.0f, dim = 0.0f;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const bool dg = (k == key);
            const float m2 = re[k] * re[k] + im[k] * im[k];
            off += dg ? 0.0f : m2;
            dre = dg ? re[k] : dre;
            dim = dg ? im[k] : dim;
        }
        *fit = finish_fitness(off, dre, dim, key >= 0, N, mode);
    }
    return ok;
}

// ----------------------------------------------------- small widths (n <= 3)
// One matrix element per lane (lane = i*N + j); a gate exchanges rows through
// a lane xor.  Lanes >= N^2 hold nothing and only exchange among themselves.
template <int NQ, bool IDENT, typename GateSrc>
__device__ __forceinline__ bool run_small_path(const float* __restrict__ T, int L, GateSrc&& src,
                                               float* U_out, FitOut* fit, int mode = QE_FIT_EQ11) {
    constexpr int N = 1 << NQ;
    constexpr bool ANG = src_angled<GateSrc>();
    using SrcT = std::decay_t<decltype(src(0))>;
    const int lane = (int)lane_id();
    const bool live = lane < N * N;
    const int i = (lane >> NQ) & (N - 1), j = lane & (N - 1);
    const SrcT dv0 = L > 0 ? src(0) : SrcT{};   // before the target: latencies overlap
    float mr = 0.0f, mi = 0.0f;
    if (live) {
        if (IDENT) {
            mr = (i == j) ? 1.0f : 0.0f;
        } else {
            const float2 v = reinterpret_cast<const float2*>(T)[(size_t)j * N + i];
            mr = v.x;
            mi = -v.y;
        }
    }
    bool ok = true;
    const float r = 0.70710678118654752f;
    const int chunks = (L + 63) >> 6;
    for (int ch = 0; ch < chunks; ++ch) {
        const SrcT dvv = ch == 0 ? dv0 : src(ch);
        const uint32_t dv = desc_of(dvv);
        const int cnt = min(64, L - ch * 64);
        const bool bad = (lane < cnt) && !desc_valid<ANG>(dv, NQ);
        if (__ballot(bad)) { ok = false; break; }
        // angled gates: lane g computes cos, sin of half of gate g's angle
        float gc = 1.0f, gs = 0.0f;
        if constexpr (ANG)
            if (lane < cnt && kind_ising((int)(dv & 15u))) half_angle(angle_of(dvv), &gc, &gs);
        for (int g = 0; g < cnt; ++g) {
            const uint32_t d = __builtin_amdgcn_readlane(dv, g);
            const int kind = d & 15;
            if (kind == KIND_I) continue;
            const int t = (d >> 4) & 15;
            const int tb = 1 << (NQ - 1 - t);
            const int mask = tb << NQ;
            const bool hi = (i & tb) != 0;
            if constexpr (ANG) {
                if (kind >= KIND_RX) {
                    const float c = bits_f(__builtin_amdgcn_readlane(f_bits(gc), g));
                    const float s = bits_f(__builtin_amdgcn_readlane(f_bits(gs), g));
                    if (kind == KIND_RZ || kind == KIND_ZZ) {
                        // diagonal: e^{-i theta/2} where the (two-wire) parity is
                        // even, e^{i theta/2} where it is odd
                        bool odd = hi;
                        if (kind == KIND_ZZ) odd = ((i >> (NQ - 1 - t)) ^ (i >> (NQ - 1 - (int)((d >> 8) & 15)))) & 1;
                        const float sg = odd ? s : -s;
                        const float br = mr, bi = mi;
                        mr = c * br - sg * bi;
                        mi = c * bi + sg * br;
                    } else {
                        const float pr = __shfl_xor(mr, mask, 64), pi = __shfl_xor(mi, mask, 64);
                        if (kind == KIND_RX) {       // c m - i s p on both rows
                            mr = c * mr + s * pi;
                            mi = c * mi - s * pr;
                        } else {                     // c m -+ s p (R_y)
                            const float sg = hi ? s : -s;
                            mr = c * mr + sg * pr;
                            mi = c * mi + sg * pi;
                        }
                    }
                    continue;
                }
            }
            const float pr = __shfl_xor(mr, mask, 64), pi = __shfl_xor(mi, mask, 64);
            bool on = true;
            if (kind_controlled(kind)) on = (i >> (NQ - 1 - ((d >> 8) & 15))) & 1;
            if (!on) continue;
            if (kind == KIND_NOT || kind == KIND_CNOT) {
                mr = pr; mi = pi;
            } else if (kind == KIND_CV || kind == KIND_CVDG) {
                // both rows of the pair: (m + p)/2 +- i (m - p)/2
                const float sr = mr + pr, si = mi + pi, dr = mr - pr, di = mi - pi;
                if (kind == KIND_CV) { mr = 0.5f * (sr - di); mi = 0.5f * (si + dr); }
                else { mr = 0.5f * (sr + di); mi = 0.5f * (si - dr); }
            } else if (kind == KIND_H) {
                const float xr = hi ? pr - mr : mr + pr, xi = hi ? pi - mi : mi + pi;
                mr = xr * r; mi = xi * r;
            } else if (hi) {   // T
                const float br = mr, bi = mi;
                mr = (br - bi) * r;
                mi = (br + bi) * r;
            }
        }
    }
    if (U_out && live) reinterpret_cast<float2*>(U_out)[(size_t)i * N + j] = make_float2(mr, mi);
    if (fit) {
        const bool dg = live && (i == j);
        const float off = (live && !dg) ? mr * mr + mi * mi : 0.0f;
        *fit = finish_fitness(off, dg ? mr : 0.0f, dg ? mi : 0.0f, dg, N, mode);
    }
    return ok;
}

// ------------------------------------------------------------ LDS-staged path
// The circuit's N x N complex64 matrix lives in LDS, row-major.  W wavefronts
// share one circuit and split its columns (CW = N / W each); since a gate only
// mixes rows, every wavefront transforms its own columns with no barrier
// between gates (LDS operations of one wavefront complete in order).  Lane l
// owns column j = w*CW + l % CW and row group rg = l / CW; pass m of a gate
// handles row pair pr = m*RG + rg (RG = 64 / CW), whose upper row index is
// the pair index with a zero (and, for a controlled gate, a one) inserted at
// the wire's bit position.  Insertion is additive over the disjoint bits of
// m*RG and rg, so a gate is described by the inserted offsets of the pair-
// index bits (rg's two bits per lane, m's bits per pass), computed for all the
// gates of a chunk at once, one gate per lane.
//
// Row relabelling: NOT and CNOT only permute rows, and the permutations they
// generate are affine maps over GF(2) of the row index.  Instead of moving
// rows, the path keeps the map phi from logical to stored rows (phi(r) =
// A r + b, A held as its columns, 6 bits each, in a 64-bit word): NOT on row
// bit p adds column p of A to b, CNOT with control bit pc and target bit pt
// adds column pt to column pc.  Every other gate addresses its logical rows
// through phi, which is linear in the pair-index bits, so its offsets are
// the images of the logical ones and combine by XOR.  The fitness reads the
// diagonal entry of column j at stored row phi(j).  (Unitary outputs keep
// the rows in place: IDENT moves them.)
__device__ __forceinline__ int ins0(int x, int pos) {
    return ((x >> pos) << (pos + 1)) | (x & ((1 << pos) - 1));
}

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Runs the circuit on this wave's columns, leaving the product in M (its
// rows under the row map, which goes to *map_out for the fitness).
// gt: this wavefront's gate table in LDS (GATE_TABLE uint4, or
// GATE_TABLE_ANGLED for angled gate sources).  NCV: the source only yields
// kinds of {I, NOT, CNOT, CV, CV+} (circuits decoded by the QEQEA sampler);
// with the row relabelling only CV and CV+ then move data, and the gate body
// needs no kind dispatch.
constexpr int GATE_TABLE = 128;
constexpr int GATE_TABLE_ANGLED = 192;

// The logical-to-stored row map of the LDS layout: logical row r of the
// product lives in stored row A r ^ b (A's column p in bits 6p..6p+5).
struct RowMap {
    uint64_t A;
    uint32_t b;
};

template <int NQ, int W, bool IDENT, bool NCV = false, typename GateSrc>
__device__ __forceinline__ bool run_lds_path(float2* M, uint4* gt, const float* __restrict__ T, int L,
                                             GateSrc&& src, RowMap* map_out, int wave = -1) {
    // CV body of one wavefront per circuit (a gate table of per-row-group
    // offsets and signs); at n = 5 each of its lanes owns two adjacent
    // columns, so that a row pair is two 16-byte accesses
    constexpr bool CVB = NCV && W == 1;
    constexpr int CPL = (CVB && NQ == 5) ? 2 : 1;          // columns per lane
    constexpr int N = 1 << NQ, CW = N / W, LPR = CW / CPL, RG = 64 / LPR;
    constexpr bool ANG = src_angled<GateSrc>();
    constexpr int ES = ANG ? 3 : 2;        // uint4 per gate-table entry
    using SrcT = std::decay_t<decltype(src(0))>;
    // four row groups per wavefront (16 columns: n = 4, or n = 5, 6 split over
    // 2 or 4 wavefronts), or two (32 columns: n = 5 in one wavefront, whose
    // half-wavefronts then read whole 256-byte rows, free of bank conflicts)
    static_assert(LPR <= 64 && 64 % LPR == 0 && N % RG == 0 && (RG == 4 || RG == 2),
                  "layout: two or four row groups per wavefront");
    static_assert((N / 2) / RG <= 8, "at most three pass bits");
    const int lane = (int)lane_id();
    if (wave < 0) wave = (int)(threadIdx.x >> 6);
    const int jl = lane % LPR, rg = lane / LPR;
    const int j = wave * CW + jl * CPL;                     // the lane's (first) column
    // The target loads are issued first, then the first chunk of descriptors
    // is fetched (or sampled, which may take dependent loads of its own), so
    // that the latencies overlap; M_0 = T^dagger (or I): M[r][j] = conj(T[j][r]).
    const float2* T2 = reinterpret_cast<const float2*>(T);
    float2 tv[CPL][N / RG];
#pragma unroll
    for (int m = 0; m < N / RG; ++m) {
        const int r = m * RG + rg;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            if (IDENT) tv[c][m] = make_float2(r == j + c ? 1.0f : 0.0f, 0.0f);
            else tv[c][m] = T2[(size_t)(j + c) * N + r];
        }
    }
    const SrcT dv0 = L > 0 ? src(0) : SrcT{};
#pragma unroll
    for (int m = 0; m < N / RG; ++m) {
        const int r = m * RG + rg;
#pragma unroll
        for (int c = 0; c < CPL; ++c)
            M[r * N + j + c] = IDENT ? tv[c][m] : make_float2(tv[c][m].x, -tv[c][m].y);
    }
    wave_lds_fence();
    bool ok = true;
    const int chunks = (L + 63) >> 6;
    // lane constants: byte offset of column j, and the row-group bits (pair
    // index bits 0 and, with four groups, 1) as all-ones / all-zeros masks
    const uint32_t jb = (uint32_t)j * 8u;
    uint32_t mb0 = (rg & 1) ? ~0u : 0u, mb1 = (rg & 2) ? ~0u : 0u;
    // as plain registers, so that selecting a gate's offset is one AND with a
    // scalar operand (a known 0 / ~0 mask becomes a move and a select)
    asm volatile("" : "+v"(mb0), "+v"(mb1));
    auto at = [&](uint32_t byte_off) -> float2& {
        return *reinterpret_cast<float2*>(reinterpret_cast<char*>(M) + byte_off);
    };
    constexpr uint32_t ROWB = NQ + 3;      // log2 of a row's byte stride (N * 8)
    constexpr bool RELABEL = !IDENT;
    // the logical-to-stored row map (wave-uniform): column p of A in bits
    // 6p..6p+5, translation b
    uint64_t Amap = 0;
#pragma unroll
    for (int p = 0; p < NQ; ++p) Amap |= (uint64_t)(1u << p) << (6 * p);
    uint32_t bmap = 0;
    // pass offsets in use: R2 from 2 passes, R3 from 4, R4 from 8 (an
    // uncontrolled gate has (N / 2) / RG passes)
    constexpr bool NIT_USES_R2 = (N / 2) / RG > 1, NIT_USES_R3 = (N / 2) / RG > 2,
                   NIT_USES_R4 = (N / 2) / RG > 4;
    // CV or CV+ of sampled NCV circuits on the lane's pairs (T0 ^ o, T0 ^ tb ^ o)
    // of column j, o over the offsets of pair-index bits 2 and 3 (o2, o3),
    // written back in place.  With a, b the two rows of a pair, p + iq = a + b
    // and u + iv = a - b, V maps (a, b) to ((p - v + i(q + u)) / 2,
    // (p + v + i(q - u)) / 2); V+ is V with u, v negated.  Each result is one
    // fused multiply-add of the exact halves p / 2, q / 2 and the exact factor
    // +-1/2 (CV +, CV+ -): it rounds (p - v) / 2 once, which is 0.5 times p - v
    // rounded.  `next` runs once the addresses are known, before the data reads.
    // With two columns per lane the same arithmetic runs on both.
    char* const Mj = reinterpret_cast<char*>(M) + jb;
    auto el = [&](uint32_t off) -> float2& { return *reinterpret_cast<float2*>(Mj + off); };
    auto el4 = [&](uint32_t off) -> float4& { return *reinterpret_cast<float4*>(Mj + off); };
    auto cv_gate = [&](const uint32_t T0, const uint32_t tb, const float hs, const uint32_t o2,
                       const uint32_t o3, auto&& next) {
        constexpr int NITC = (N / 4) / RG;
        const uint32_t T1 = T0 ^ tb;
        uint32_t offm[NITC];
        offm[0] = 0u;
        if constexpr (NITC > 1) offm[1] = o2;
        if constexpr (NITC > 2) { offm[2] = o3; offm[3] = o2 ^ o3; }
        next();
        if constexpr (CPL == 2) {
            float4 A[NITC], B[NITC];
#pragma unroll
            for (int m = 0; m < NITC; ++m) { A[m] = el4(T0 ^ offm[m]); B[m] = el4(T1 ^ offm[m]); }
#pragma unroll
            for (int m = 0; m < NITC; ++m) {
                const float4 a = A[m], b = B[m];
                const float ph0 = 0.5f * (a.x + b.x), qh0 = 0.5f * (a.y + b.y), u0 = a.x - b.x, v0 = a.y - b.y;
                const float ph1 = 0.5f * (a.z + b.z), qh1 = 0.5f * (a.w + b.w), u1 = a.z - b.z, v1 = a.w - b.w;
                el4(T0 ^ offm[m]) = make_float4(__builtin_fmaf(hs, -v0, ph0), __builtin_fmaf(hs, u0, qh0),
                                                __builtin_fmaf(hs, -v1, ph1), __builtin_fmaf(hs, u1, qh1));
                el4(T1 ^ offm[m]) = make_float4(__builtin_fmaf(hs, v0, ph0), __builtin_fmaf(hs, -u0, qh0),
                                                __builtin_fmaf(hs, v1, ph1), __builtin_fmaf(hs, -u1, qh1));
            }
        } else {
            float2 A[NITC], B[NITC];
#pragma unroll
            for (int m = 0; m < NITC; ++m) { A[m] = el(T0 ^ offm[m]); B[m] = el(T1 ^ offm[m]); }
#pragma unroll
            for (int m = 0; m < NITC; ++m) {
                const float2 a = A[m], b = B[m];
                const float ph = 0.5f * (a.x + b.x), qh = 0.5f * (a.y + b.y), u = a.x - b.x, v = a.y - b.y;
                el(T0 ^ offm[m]) = make_float2(__builtin_fmaf(hs, -v, ph), __builtin_fmaf(hs, u, qh));
                el(T1 ^ offm[m]) = make_float2(__builtin_fmaf(hs, v, ph), __builtin_fmaf(hs, -u, qh));
            }
        }
    };
    for (int ch = 0; ch < chunks; ++ch) {
        const SrcT dvv = ch == 0 ? dv0 : src(ch);
        const uint32_t dv = desc_of(dvv);
        const int cnt = min(64, L - ch * 64);
        const bool bad = (lane < cnt) && !desc_valid<ANG>(dv, NQ);
        if (__ballot(bad)) { ok = false; break; }
        // Gate program: each lane computes the constants of its own gate (lane
        // g: gate g of the chunk): the byte offsets in M of pair-index bits
        // 0..4 once the target bit (and the control bit) are inserted as
        // zeros, the control row offset and the partner row offset.  With one
        // wavefront per circuit (W = 1) the non-identity gates are packed in
        // order into this wave's LDS table (two uint4 per gate), which the
        // loop reads with broadcast loads one gate ahead; with W > 1 (LDS
        // bandwidth is the bound there) the loop reads them from the lanes
        // with v_readlane, visiting the set bits of a ballot of non-identity
        // gates.  Angled gates add a third word pair: cos and sin of half the
        // gate's angle.  The interaction inserts both of its wires' bits like
        // a controlled gate; its "control" offset is its second wire.
        const int kind = (int)(dv & 15u);
        const int tpos = NQ - 1 - (int)((dv >> 4) & 15u);
        const int cpos = NQ - 1 - (int)((dv >> 8) & 15u);
        const bool ctl = kind_two_wire(kind);
        const int lo = ctl ? min(tpos, cpos) : tpos, hi = ctl ? max(tpos, cpos) : tpos;
        const bool perm = RELABEL && (kind == KIND_NOT || kind == KIND_CNOT);
        // fold this chunk's NOT / CNOT into the row map, in circuit order; each
        // lane keeps the map in force at its own gate
        uint64_t myA = Amap;
        uint32_t myB = bmap;
        if constexpr (RELABEL) {
            uint64_t pm = __ballot(lane < cnt && perm);
            while (pm) {
                const int g = (int)__builtin_ctzll(pm);
                pm &= pm - 1;
                const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)dv, g);
                const int pt = NQ - 1 - (int)((d >> 4) & 15u);
                const uint32_t colt = (uint32_t)(Amap >> (6 * pt)) & 63u;
                if ((d & 15u) == (uint32_t)KIND_NOT) {
                    bmap ^= colt;
                } else {
                    const int pc = NQ - 1 - (int)((d >> 8) & 15u);
                    Amap ^= (uint64_t)colt << (6 * pc);
                }
                if (lane > g) { myA = Amap; myB = bmap; }
            }
        }
        // stored byte offset of logical row bit q under the lane's map
        auto colb = [&](int q) -> uint32_t { return ((uint32_t)(myA >> (6 * q)) & 63u) << ROWB; };
        // insertion of the gate's zero bits, then the image of the single
        // logical row bit that pair-index bit x lands on
        auto ins = [&](int x) -> uint32_t {
            int y = ins0(x, lo);
            if (ctl) y = ins0(y, hi);
            return colb(__builtin_ctz((uint32_t)y));
        };
        const bool live = lane < cnt && kind != KIND_I && !perm;
        const uint64_t live_mask = __ballot(live);
        // the row group selects pair-index bits 0 (and 1); the passes walk
        // the pair-index bits above them
        const uint4 G0 = make_uint4(ins(1), RG == 4 ? ins(2) : 0u, ctl ? colb(cpos) : 0u, colb(tpos));
        const uint4 G1 = make_uint4((uint32_t)kind | ((myB << ROWB) << 16), NIT_USES_R2 ? ins(RG) : 0u,
                                    NIT_USES_R3 ? ins(2 * RG) : 0u, NIT_USES_R4 ? ins(4 * RG) : 0u);
        uint4 G2 = make_uint4(f_bits(1.0f), 0u, 0u, 0u);
        if constexpr (ANG) {
            if (live && kind_ising(kind)) {
                float gc, gs;
                half_angle(angle_of(dvv), &gc, &gs);
                G2 = make_uint4(f_bits(gc), f_bits(gs), 0u, 0u);
            }
        }
        // one gate from its table entry (E0, E1, E2); `next` issues the load
        // of the following entry once the addresses are known and before the
        // data reads, so the entry is ready when its gate starts
        auto apply = [&](const uint4 E0, const uint4 E1, const uint4 E2, auto&& next) {
            const uint32_t kx = (uint32_t)__builtin_amdgcn_readfirstlane((int)E1.x);
            const int k = (int)(kx & 15u);
            // the row group's pair bits and the map's translation
            const uint32_t rgo = (mb0 & E0.x) ^ (mb1 & E0.y) ^ (kx >> 16);
            const uint32_t tb = E0.w;
            next();
            if constexpr (ANG) {
                if (k >= KIND_RX) {
                    const float c = bits_f(E2.x), s = bits_f(E2.y);
                    if (k == KIND_ZZ) {
                        // diagonal: rows whose two wire bits agree take
                        // e^{-i theta/2}, the others e^{i theta/2}
                        constexpr int NIT = (N / 4) / RG;
                        uint32_t offm[NIT];
                        offm[0] = 0u;
                        if constexpr (NIT > 1) offm[1] = E1.y;
                        if constexpr (NIT > 2) { offm[2] = E1.z; offm[3] = E1.y ^ E1.z; }
                        const uint32_t a0 = rgo ^ jb, cb = E0.z;
                        float2 X[NIT][4];
#pragma unroll
                        for (int m = 0; m < NIT; ++m) {
                            X[m][0] = at(a0 ^ offm[m]);
                            X[m][1] = at(a0 ^ cb ^ offm[m]);
                            X[m][2] = at(a0 ^ tb ^ offm[m]);
                            X[m][3] = at(a0 ^ cb ^ tb ^ offm[m]);
                        }
#pragma unroll
                        for (int m = 0; m < NIT; ++m) {
                            at(a0 ^ offm[m]) = phase_minus(X[m][0], c, s);
                            at(a0 ^ cb ^ offm[m]) = phase_plus(X[m][1], c, s);
                            at(a0 ^ tb ^ offm[m]) = phase_plus(X[m][2], c, s);
                            at(a0 ^ cb ^ tb ^ offm[m]) = phase_minus(X[m][3], c, s);
                        }
                        return;
                    }
                    constexpr int NIT = (N / 2) / RG;
                    uint32_t offm[NIT];
                    offm[0] = 0u;
                    if constexpr (NIT > 1) offm[1] = E1.y;
                    if constexpr (NIT > 2) { offm[2] = E1.z; offm[3] = E1.y ^ E1.z; }
                    if constexpr (NIT > 4) {
#pragma unroll
                        for (int m = 4; m < 8; ++m) offm[m] = offm[m - 4] ^ E1.w;
                    }
                    const uint32_t a0 = rgo ^ jb, a1 = a0 ^ tb;
                    float2 A[NIT], B[NIT];
#pragma unroll
                    for (int m = 0; m < NIT; ++m) { A[m] = at(a0 ^ offm[m]); B[m] = at(a1 ^ offm[m]); }
                    if (k == KIND_RZ) {
#pragma unroll
                        for (int m = 0; m < NIT; ++m) {
                            at(a0 ^ offm[m]) = phase_minus(A[m], c, s);
                            at(a1 ^ offm[m]) = phase_plus(B[m], c, s);
                        }
                    } else if (k == KIND_RX) {   // a' = c a - i s b, b' = c b - i s a
#pragma unroll
                        for (int m = 0; m < NIT; ++m) {
                            const float2 a = A[m], b = B[m];
                            at(a0 ^ offm[m]) = make_float2(c * a.x + s * b.y, c * a.y - s * b.x);
                            at(a1 ^ offm[m]) = make_float2(c * b.x + s * a.y, c * b.y - s * a.x);
                        }
                    } else {                     // R_y: a' = c a - s b, b' = s a + c b
#pragma unroll
                        for (int m = 0; m < NIT; ++m) {
                            const float2 a = A[m], b = B[m];
                            at(a0 ^ offm[m]) = make_float2(c * a.x - s * b.x, c * a.y - s * b.y);
                            at(a1 ^ offm[m]) = make_float2(s * a.x + c * b.x, s * a.y + c * b.y);
                        }
                    }
                    return;
                }
            }
            static_assert(!NCV || (RELABEL && !ANG), "the NCV body needs the relabelling");
            if (NCV || (k >= KIND_CNOT && k <= KIND_CVDG)) {
                constexpr int NIT = (N / 4) / RG;
                uint32_t offm[NIT];
                offm[0] = 0u;
                if constexpr (NIT > 1) offm[1] = E1.y;
                if constexpr (NIT > 2) { offm[2] = E1.z; offm[3] = E1.y ^ E1.z; }
                const uint32_t a0 = rgo ^ jb ^ E0.z, a1 = a0 ^ tb;
                float2 A[NIT], B[NIT];
#pragma unroll
                for (int m = 0; m < NIT; ++m) { A[m] = at(a0 ^ offm[m]); B[m] = at(a1 ^ offm[m]); }
                // (with the row relabelling, NOT and CNOT never get here)
                if (!RELABEL && !NCV && k == KIND_CNOT) {
#pragma unroll
                    for (int m = 0; m < NIT; ++m) { at(a0 ^ offm[m]) = B[m]; at(a1 ^ offm[m]) = A[m]; }
                } else {
                    // CV: (a, b) -> V (a, b); CV+ is CV with a - b negated: one
                    // fused multiply-add of the exact halves and the factor
                    // +-1/2 per result, as in the CV body of sampled circuits
                    const float hs = k == KIND_CVDG ? -0.5f : 0.5f;
#pragma unroll
                    for (int m = 0; m < NIT; ++m) {
                        const float2 a = A[m], b = B[m];
                        const float ph = 0.5f * (a.x + b.x), qh = 0.5f * (a.y + b.y), u = a.x - b.x,
                                    v = a.y - b.y;
                        at(a0 ^ offm[m]) = make_float2(__builtin_fmaf(hs, -v, ph), __builtin_fmaf(hs, u, qh));
                        at(a1 ^ offm[m]) = make_float2(__builtin_fmaf(hs, v, ph), __builtin_fmaf(hs, -u, qh));
                    }
                }
            } else {
                constexpr int NIT = (N / 2) / RG;
                uint32_t offm[NIT];
                offm[0] = 0u;
                if constexpr (NIT > 1) offm[1] = E1.y;
                if constexpr (NIT > 2) { offm[2] = E1.z; offm[3] = E1.y ^ E1.z; }
                if constexpr (NIT > 4) {
#pragma unroll
                    for (int m = 4; m < 8; ++m) offm[m] = offm[m - 4] ^ E1.w;
                }
                const uint32_t a0 = rgo ^ jb, a1 = a0 ^ tb;
                const float r = 0.70710678118654752f;
                if (k == KIND_T) {
#pragma unroll
                    for (int m = 0; m < NIT; ++m) {
                        const float2 b = at(a1 ^ offm[m]);
                        at(a1 ^ offm[m]) = make_float2((b.x - b.y) * r, (b.x + b.y) * r);
                    }
                } else {
                    float2 A[NIT], B[NIT];
#pragma unroll
                    for (int m = 0; m < NIT; ++m) { A[m] = at(a0 ^ offm[m]); B[m] = at(a1 ^ offm[m]); }
                    if (!RELABEL && k == KIND_NOT) {
#pragma unroll
                        for (int m = 0; m < NIT; ++m) { at(a0 ^ offm[m]) = B[m]; at(a1 ^ offm[m]) = A[m]; }
                    } else {   // H
#pragma unroll
                        for (int m = 0; m < NIT; ++m) {
                            const float2 a = A[m], b = B[m];
                            at(a0 ^ offm[m]) = make_float2((a.x + b.x) * r, (a.y + b.y) * r);
                            at(a1 ^ offm[m]) = make_float2((a.x - b.x) * r, (a.y - b.y) * r);
                        }
                    }
                }
            }
        };
        if constexpr (CVB) {
            // Only CV and CV+ move data (NOT and CNOT live in the row map).
            // Entry e of the table: words 0..3 hold, for row group rg, the
            // stored byte offset of the first row of the group's pair (pair
            // index bits 0, 1 = rg inserted, the control row and the map's
            // translation folded in), so that a lane reads its own word; then
            // the target row offset, the signed half (CV: 1/2, CV+: -1/2) and
            // the offsets of pair-index bits 2 and 3.
            constexpr int NITC = (N / 4) / RG;
            const int count = __popcll(live_mask);
            if (live) {
                const int rank = (int)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(live_mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)live_mask, 0u));
                const uint32_t base = (myB << ROWB) ^ colb(cpos), i1 = ins(1), i2 = RG == 4 ? ins(2) : 0u;
                gt[2 * rank] = make_uint4(base, base ^ i1, base ^ i2, base ^ i1 ^ i2);
                gt[2 * rank + 1] = make_uint4(colb(tpos), f_bits(kind == KIND_CVDG ? -0.5f : 0.5f),
                                              NITC > 1 ? ins(RG) : 0u, NITC > 2 ? ins(2 * RG) : 0u);
            }
            wave_lds_fence();
            const uint32_t* gw = reinterpret_cast<const uint32_t*>(gt) + rg;   // entry 0, this row group
            auto cv = [&](const uint32_t T0, const uint4 E, auto&& next) {
                cv_gate(T0, E.x, bits_f(E.y), E.z, E.w, next);
            };
            // whole pairs of gates per iteration (no exit test between them),
            // each entry loaded one gate ahead; the second prefetch is clamped
            // to the last entry, and an odd last gate runs after the loop
            uint32_t ta = 0u, tb2 = 0u;
            uint4 ea = make_uint4(0u, 0u, 0u, 0u), eb = ea;
            if (count > 0) { ta = gw[0]; ea = gt[1]; }
            // lgkmcnt(0): the first entry is in place before the loop, so that
            // inside it only the data reads are waited for (the entry of the
            // next gate is issued ahead of them and arrives first)
            __builtin_amdgcn_s_waitcnt(0xC07F);
            int e = 0;
            for (; e + 2 <= count; e += 2) {
                cv(ta, ea, [&] { tb2 = gw[8 * (e + 1)]; eb = gt[2 * (e + 1) + 1]; });
                wave_lds_fence();
                const int e2 = min(e + 2, count - 1);
                cv(tb2, eb, [&] { ta = gw[8 * e2]; ea = gt[2 * e2 + 1]; });
                wave_lds_fence();
            }
            if (e < count) {
                cv(ta, ea, [] {});
                wave_lds_fence();
            }
        } else if constexpr (W == 1) {
            const int count = __popcll(live_mask);
            if (live) {
                const int rank = (int)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(live_mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)live_mask, 0u));
                gt[ES * rank] = G0;
                gt[ES * rank + 1] = G1;
                if constexpr (ANG) gt[ES * rank + 2] = G2;
            }
            wave_lds_fence();
            // whole pairs of gates per iteration, each entry loaded one gate
            // ahead (the unrolled pair keeps the prefetched entries in place;
            // the second prefetch is clamped to the last entry, an odd last
            // gate runs after the loop)
            uint4 a0e = make_uint4(0u, 0u, 0u, 0u), a1e = a0e, a2e = a0e, b0e = a0e, b1e = a0e, b2e = a0e;
            auto fetch = [&](int e, uint4& x0, uint4& x1, uint4& x2) {
                x0 = gt[ES * e];
                x1 = gt[ES * e + 1];
                if constexpr (ANG) x2 = gt[ES * e + 2];
            };
            if (count > 0) fetch(0, a0e, a1e, a2e);
            int e = 0;
            for (; e + 2 <= count; e += 2) {
                apply(a0e, a1e, a2e, [&] { fetch(e + 1, b0e, b1e, b2e); });
                wave_lds_fence();
                const int e2 = min(e + 2, count - 1);
                apply(b0e, b1e, b2e, [&] { fetch(e2, a0e, a1e, a2e); });
                wave_lds_fence();
            }
            if (e < count) {
                apply(a0e, a1e, a2e, [] {});
                wave_lds_fence();
            }
        } else if constexpr (NCV) {
            // W > 1: the CV body with each gate's constants read from the lane
            // that owns it (the row group's offset from the base and the
            // offsets of pair-index bits 0, 1; the sign in the target word's
            // top bit, free since offsets stay below 2^15)
            (void)gt;
            constexpr int NITC = (N / 4) / RG;
            const uint32_t gbase = (myB << ROWB) ^ colb(cpos), gi1 = ins(1), gi2 = RG == 4 ? ins(2) : 0u;
            const uint32_t gtw = colb(tpos) | (kind == KIND_CVDG ? 0x80000000u : 0u);
            const uint32_t go2 = NITC > 1 ? ins(RG) : 0u, go3 = NITC > 2 ? ins(2 * RG) : 0u;
            uint64_t todo = live_mask;
            while (todo) {
                const int g = (int)__builtin_ctzll(todo);
                todo &= todo - 1;
                auto rl = [&](uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, g); };
                const uint32_t T0 = rl(gbase) ^ (mb0 & rl(gi1)) ^ (mb1 & rl(gi2));
                const uint32_t tw = rl(gtw);
                cv_gate(T0, tw & 0x7FFFFFFFu, (tw >> 31) ? -0.5f : 0.5f, NITC > 1 ? rl(go2) : 0u,
                        NITC > 2 ? rl(go3) : 0u, [] {});
                wave_lds_fence();
            }
        } else {
            (void)gt;
            uint64_t todo = live_mask;
            while (todo) {
                const int g = (int)__builtin_ctzll(todo);
                todo &= todo - 1;
                auto rl = [&](uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, g); };
                const uint4 E0 = make_uint4(rl(G0.x), rl(G0.y), rl(G0.z), rl(G0.w));
                const uint4 E1 = make_uint4(rl(G1.x), NIT_USES_R2 ? rl(G1.y) : 0u,
                                            NIT_USES_R3 ? rl(G1.z) : 0u, NIT_USES_R4 ? rl(G1.w) : 0u);
                const uint4 E2 = ANG ? make_uint4(rl(G2.x), rl(G2.y), 0u, 0u) : G2;
                apply(E0, E1, E2, [] {});
                wave_lds_fence();
            }
        }
    }
    if (map_out) *map_out = RowMap{Amap, bmap};
    return ok;
}

// ----------------------------------------------------- generic LDS body
// One workgroup of 256 threads per circuit, any width 1..6, any precision:
// M lives in LDS and every gate is one pass over the row pairs it touches,
// followed by a workgroup barrier.  The FP64 instance re-checks elite
// circuits and builds FP64 target unitaries; the FP32 one cross-checks the
// tuned kernels.  err != 0 on entry: the circuit is malformed and only NaN is
// written.  Outputs (f, g, delta: one element; U: N*N complex) may be null.
template <typename Real>
struct Cplx {
    Real r, i;
};

template <typename Real>
__device__ __forceinline__ void gate_coeffs(int kind, Cplx<Real> G[4]) {
    const Real h = (Real)0.5, z = (Real)0, o = (Real)1;
    const Real s = (Real)0.70710678118654752440084436210485;
    switch (kind) {
        case KIND_NOT: case KIND_CNOT:
            G[0] = {z, z}; G[1] = {o, z}; G[2] = {o, z}; G[3] = {z, z}; break;
        case KIND_CV:
            G[0] = {h, h}; G[1] = {h, -h}; G[2] = {h, -h}; G[3] = {h, h}; break;
        case KIND_CVDG:
            G[0] = {h, -h}; G[1] = {h, h}; G[2] = {h, h}; G[3] = {h, -h}; break;
        case KIND_H:
            G[0] = {s, z}; G[1] = {s, z}; G[2] = {s, z}; G[3] = {-s, z}; break;
        default:   // T
            G[0] = {o, z}; G[1] = {z, z}; G[2] = {z, z}; G[3] = {s, s}; break;
    }
}

// Coefficients [[G0, G1], [G2, G3]] of a rotation (Eqs. 3-5) from c, s =
// cos, sin of half its angle.
template <typename Real>
__device__ __forceinline__ void rotation_coeffs(int kind, Real c, Real s, Cplx<Real> G[4]) {
    const Real z = (Real)0;
    if (kind == KIND_RX) {
        G[0] = {c, z}; G[1] = {z, -s}; G[2] = {z, -s}; G[3] = {c, z};
    } else if (kind == KIND_RY) {
        G[0] = {c, z}; G[1] = {-s, z}; G[2] = {s, z}; G[3] = {c, z};
    } else {   // R_z
        G[0] = {c, -s}; G[1] = {z, z}; G[2] = {z, z}; G[3] = {c, s};
    }
}

template <typename Real>
__device__ __forceinline__ Real block_sum(Real v, Real* scratch) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    Real t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += scratch[k];
    return t;
}

// Eq. 11 (or the phase-insensitive fitness) of the N x N matrix M held in
// LDS as separate real / imaginary arrays, reduced over the workgroup.  ok
// false: the circuit was malformed (err says why) and NaN is written.
// red: 8 values of LDS scratch.  Every thread of the workgroup must call it.
template <typename Real>
__device__ __forceinline__ void lds_fitness(const Real* Mr, const Real* Mi, int N, bool ok, uint32_t err,
                                            Real* f, Real* g, Real* delta, uint32_t* errw, int mode,
                                            Real* red) {
    const int tid = threadIdx.x, nt = blockDim.x, NN = N * N;
    const Real nan = (Real)__builtin_nan("");
    Real off = 0, tr = 0, ti = 0;
    if (ok) {
        for (int e = tid; e < NN; e += nt) {
            const int i = e / N, j = e - i * N;
            if (i == j) { tr += Mr[e]; ti += Mi[e]; }
            else off += Mr[e] * Mr[e] + Mi[e] * Mi[e];
        }
    }
    tr = block_sum(tr, red);
    ti = block_sum(ti, red);
    off = block_sum(off, red);
    const Real am = sqrt(tr * tr + ti * ti);
    Real er = 1, ei = 0;
    if (am > 0) { er = tr / am; ei = ti / am; }
    Real D = 0;
    if (ok)
        for (int i = tid; i < N; i += nt) {
            const Real xr = Mr[i * N + i] - er, xi = Mi[i * N + i] - ei;
            D += xr * xr + xi * xi;
        }
    D = block_sum(D, red);
    if (tid == 0) {
        Real fv, gv, dl;
        if (mode == QE_FIT_PHASE_INSENSITIVE) {
            fitness_pi(off, N, &fv, &gv, &dl);
        } else {
            dl = (Real)0.5 * (off + D);
            Real q = dl / (Real)N;
            q = q < 0 ? (Real)0 : (q > 1 ? (Real)1 : q);
            fv = (Real)1 - sqrt(q);
            gv = am / (Real)N;
        }
        if (ok && !(fv == fv)) err = QE_DEVERR_NUMERIC;
        if (f) *f = ok ? fv : nan;
        if (g) *g = ok ? gv : nan;
        if (delta) *delta = ok ? dl : nan;
        if (err) atomicOr(errw, err);
    }
}

// Dynamic LDS of the generic-body kernels: two planes of 4^n reals.
template <typename Real>
__device__ __forceinline__ Real* generic_lds() {
    extern __shared__ __align__(16) unsigned char qe_generic_lds[];
    return reinterpret_cast<Real*>(qe_generic_lds);
}
__host__ __device__ inline size_t generic_lds_bytes(int n, size_t real_bytes) {
    return (size_t)2 * ((size_t)1 << (2 * n)) * real_bytes;
}

// angles: the gates' angles (u32 turn fractions, parallel to gates) or
// NULL, in which case the Ising kinds are invalid descriptors.  Mr, Mi: LDS
// for the real and imaginary parts of the 2^n x 2^n matrix (the caller sizes
// them for its widths).
template <typename Real, bool IDENT>
__device__ __forceinline__ void lds_generic_body(int n, int L, const uint16_t* gates,
                                                 const uint32_t* angles, const Real* T, uint32_t err,
                                                 Real* f, Real* g, Real* delta, Real* U,
                                                 uint32_t* errw, int mode, Real* Mr, Real* Mi) {
    __shared__ Real red[8];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lg = err == QE_DEVERR_WIDTH ? 1 : n;     // log2 of the matrix size
    const int N = 1 << lg;
    const int NN = N * N;
    bool ok = err == 0;
    if (ok) {
        for (int e = tid; e < NN; e += nt) {
            const int i = e >> lg, j = e & (N - 1);
            if (IDENT) {
                Mr[e] = (i == j) ? (Real)1 : (Real)0;
                Mi[e] = 0;
            } else {
                Mr[e] = T[2 * ((size_t)j * N + i)];
                Mi[e] = -T[2 * ((size_t)j * N + i) + 1];
            }
        }
        __syncthreads();
        for (int l = 0; l < L; ++l) {
            const uint32_t d = gates[l];
            if (angles ? !desc_valid<true>(d, n) : !desc_valid(d, n)) { ok = false; break; }
            const int kind = d & 15;
            if (kind == KIND_I) continue;
            const int tpos = n - 1 - (int)((d >> 4) & 15);
            const int tb = 1 << tpos;
            Cplx<Real> G[4];
            if (kind_ising(kind)) {
                Real c, s;
                half_angle(angles[l], &c, &s);
                if (kind == KIND_ZZ) {
                    // diagonal: e^{-i theta/2} where the two wire bits agree,
                    // e^{i theta/2} where they differ
                    const int cpos = n - 1 - (int)((d >> 8) & 15);
                    for (int e = tid; e < NN; e += nt) {
                        const int i = e >> lg;
                        const Real sg = (((i >> tpos) ^ (i >> cpos)) & 1) ? s : -s;
                        const Real ar = Mr[e], ai = Mi[e];
                        Mr[e] = c * ar - sg * ai;
                        Mi[e] = c * ai + sg * ar;
                    }
                    __syncthreads();
                    continue;
                }
                rotation_coeffs<Real>(kind, c, s, G);
            } else {
                gate_coeffs<Real>(kind, G);
            }
            const int cb = kind_controlled(kind) ? 1 << (n - 1 - (int)((d >> 8) & 15)) : 0;
            for (int e = tid; e < NN / 2; e += nt) {
                const int p = e >> lg, j = e & (N - 1);
                const int i0 = ((p >> tpos) << (tpos + 1)) | (p & (tb - 1));
                if (cb && !(i0 & cb)) continue;
                const int i1 = i0 | tb;
                const Real ar = Mr[i0 * N + j], ai = Mi[i0 * N + j];
                const Real br = Mr[i1 * N + j], bi = Mi[i1 * N + j];
                Mr[i0 * N + j] = G[0].r * ar - G[0].i * ai + G[1].r * br - G[1].i * bi;
                Mi[i0 * N + j] = G[0].r * ai + G[0].i * ar + G[1].r * bi + G[1].i * br;
                Mr[i1 * N + j] = G[2].r * ar - G[2].i * ai + G[3].r * br - G[3].i * bi;
                Mi[i1 * N + j] = G[2].r * ai + G[2].i * ar + G[3].r * bi + G[3].i * br;
            }
            __syncthreads();
        }
        if (!ok) err = QE_DEVERR_DESC;
    }
    const Real nan = (Real)__builtin_nan("");
    if (IDENT) {
        if (U)
            for (int e = tid; e < NN; e += nt) {
                U[2 * e] = ok ? Mr[e] : nan;
                U[2 * e + 1] = ok ? Mi[e] : nan;
            }
        if (tid == 0 && err) atomicOr(errw, err);
        return;
    }
    lds_fitness<Real>(Mr, Mi, N, ok, err, f, g, delta, errw, mode, red);
}

// Eq. 11 (or the phase-insensitive form) of one circuit from its product in
// LDS, in an order fixed by the width alone.  WR wavefronts share the work
// (WR = 1 for widths up to 5, whose kernels may run one or two wavefronts per
// circuit; WR = 4 for width 6, whose kernels all run four): lane l of
// wavefront w takes column j = w (N / WR) + l mod (N / WR) and the logical
// rows r = q, q + Q, q + 2Q, ... (q = l div (N / WR), Q = 64 WR / N) in
// increasing order (row r is stored at A r ^ b); the wavefront's reduction
// tree adds its lanes and the WR wavefront sums are added in order.  Every
// LDS-staged schedule of a width therefore gives the same bits.  WR > 1:
// every wavefront of the circuit calls it (it holds workgroup barriers) with
// `w` its index and red 4 x 3 floats of LDS.  Returns f on every lane; g,
// delta out.
template <int NQ, int WR>
__device__ __forceinline__ float canonical_fitness(const float2* M, const RowMap map, int mode,
                                                   float* g_out, float* delta_out, int w = 0,
                                                   float (*red)[3] = nullptr) {
    constexpr int N = 1 << NQ, CWR = N / WR, Q = 64 / CWR, ROWB = NQ + 3;
    static_assert(CWR <= 64 && 64 % CWR == 0 && Q <= N, "reduction layout");
    const int lane = (int)lane_id(), j = w * CWR + lane % CWR, q = lane / CWR;
    const char* Mj = reinterpret_cast<const char*>(M) + (uint32_t)j * 8u;
    auto col = [&](int p) -> uint32_t { return (uint32_t)(map.A >> (6 * p)) & 63u; };
    // stored row of logical row q (lane part) and of Q m (uniform part)
    uint32_t sq = 0u;
#pragma unroll
    for (int p = 0; p < NQ; ++p)
        if ((1 << p) < Q && ((q >> p) & 1)) sq ^= col(p);
    // the rows in blocks of at most 16 (the block's reads are issued together)
    constexpr int R = N / Q, BLK = R < 16 ? R : 16;
    float off = 0.0f;
    float2 d = make_float2(0.0f, 0.0f);
    for (int m0 = 0; m0 < R; m0 += BLK) {
        uint32_t s0 = map.b;               // stored image of Q m0 (bits above the block's)
#pragma unroll
        for (int p = 0; p < NQ; ++p)
            if (((Q * m0) >> p) & 1) s0 ^= col(p);
        float2 v[BLK];
#pragma unroll
        for (int i = 0; i < BLK; ++i) {
            uint32_t sm = s0;
#pragma unroll
            for (int p = 0; p < NQ; ++p)
                if (((Q * i) >> p) & 1) sm ^= col(p);
            v[i] = *reinterpret_cast<const float2*>(Mj + ((sq ^ sm) << ROWB));
        }
        // (the reads stay unconditional: under the diagonal test each would
        // be waited for in turn)
#pragma unroll
        for (int i = 0; i < BLK; ++i) asm volatile("" ::"v"(v[i].x), "v"(v[i].y));
#pragma unroll
        for (int i = 0; i < BLK; ++i) {
            const int r = q + Q * (m0 + i);
            if (r == j) d = v[i];
            else off += v[i].x * v[i].x + v[i].y * v[i].y;
        }
    }
    // sums over the circuit's WR wavefronts, added in order
    auto total = [&](float x) -> float {
        const float s = wave_sum(x);
        if constexpr (WR == 1) {
            return s;
        } else {
            __syncthreads();
            if (lane == 0) red[w][0] = s;
            __syncthreads();
            float t = 0.0f;
#pragma unroll
            for (int k = 0; k < WR; ++k) t += red[k][0];
            return t;
        }
    };
    const float offs = total(off);
    if (mode == QE_FIT_PHASE_INSENSITIVE) {
        float fv;
        fitness_pi(offs, N, &fv, g_out, delta_out);
        return fv;
    }
    const float tr = total(d.x), ti = total(d.y);
    const float am = sqrtf(tr * tr + ti * ti);
    float er = 1.0f, ei = 0.0f;
    if (am > 0.0f) { er = tr / am; ei = ti / am; }
    float dl = 0.0f;
    if (j % Q == q) { const float xr = d.x - er, xi = d.y - ei; dl = xr * xr + xi * xi; }
    const float dlt = 0.5f * (offs + total(dl));
    const float qq = fminf(fmaxf(dlt / (float)N, 0.0f), 1.0f);
    *g_out = am / (float)N;
    *delta_out = dlt;
    return 1.0f - sqrtf(qq);
}

// wavefronts of the canonical reduction per width
template <int NQ>
constexpr int reduction_waves() { return NQ == 6 ? 4 : 1; }

template <bool IDENT, typename GateSrc>
__device__ __forceinline__ bool run_any_width(int n, const float* __restrict__ T, int L,
                                              GateSrc&& src, float* U_out, FitOut* fit, int mode) {
    switch (n) {
        case 1: return run_small_path<1, IDENT>(T, L, src, U_out, fit, mode);
        case 2: return run_small_path<2, IDENT>(T, L, src, U_out, fit, mode);
        case 3: return run_small_path<3, IDENT>(T, L, src, U_out, fit, mode);
        case 4: return run_register_path<4, IDENT>(T, L, src, U_out, fit, mode);
        case 5: return run_register_path<5, IDENT>(T, L, src, U_out, fit, mode);
        default: return run_register_path<6, IDENT>(T, L, src, U_out, fit, mode);
    }
}

template <int NQ, bool IDENT, typename GateSrc>
__device__ __forceinline__ bool run_width(int n, const float* __restrict__ T, int L, GateSrc&& src,
                                          float* U_out, FitOut* fit, int mode = QE_FIT_EQ11) {
    if constexpr (NQ == 0) return run_any_width<IDENT>(n, T, L, src, U_out, fit, mode);
    else if constexpr (NQ <= 3) return run_small_path<NQ, IDENT>(T, L, src, U_out, fit, mode);
    else return run_register_path<NQ, IDENT>(T, L, src, U_out, fit, mode);
}

}  // namespace qe
