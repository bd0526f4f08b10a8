// Batched circuit-fitness kernels (Eq. 11 of Sec. IV-E) and unitary builders.
#include "../../include/qe.h"
#include "qe_eval_core.hpp"
#include "qe_internal.hpp"

namespace qe {

constexpr int WPB = 4;   // wavefronts (circuits) per workgroup

__device__ __forceinline__ Item resolve(const BatchArgs& a, int b, bool need_target = true) {
    return resolve_item(a, b, need_target);
}

// Gate p of a circuit as its gate source returns it: the descriptor, or
// with ANG the descriptor and its angle (0 beyond the circuit).
template <bool ANG>
__device__ __forceinline__ auto batch_gate(const Item& it, int p) {
    if constexpr (ANG)
        return p < it.L ? make_uint2((uint32_t)it.g[p], it.ang[p]) : make_uint2(0u, 0u);
    else
        return p < it.L ? (uint32_t)it.g[p] : 0u;
}

// ------------------------------------------------------- FP32, one wave each
// Register-resident path (n = 4..6) or one-element-per-lane path (n <= 3);
// WPB circuits per workgroup.  FILTER: a mixed-width batch is served by one
// launch per width, each skipping the circuits of other widths.  ANG: the
// batch carries angles (one-element-per-lane path only).
template <int NQ, bool FILTER, bool ANG = false>
__global__ __launch_bounds__(64 * WPB) void wave_kernel(BatchArgs a, float* __restrict__ f,
                                                        float* __restrict__ g,
                                                        float* __restrict__ delta) {
    const int b = __builtin_amdgcn_readfirstlane(blockIdx.x * WPB + (threadIdx.x >> 6));
    if (b >= a.B) return;
    const int lane = (int)lane_id();
    Item it = resolve(a, b);
    if (FILTER && it.n != NQ) return;
    if (it.err == 0 && it.n != NQ) it.err = QE_DEVERR_WIDTH;
    FitOut o{__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
    if (it.err == 0) {
        const int L = it.L;
        auto src = [&](int ch) { return batch_gate<ANG>(it, ch * 64 + lane); };
        const float* T = reinterpret_cast<const float*>(a.targets) + 2 * it.toff;
        static_assert(!ANG || NQ <= 3, "angled circuits of 4 or more wires take the LDS-staged path");
        const bool ok = run_width<NQ, false>(NQ, T, L, src, nullptr, &o, a.mode);
        if (!ok) {
            it.err = QE_DEVERR_DESC;
            o = FitOut{__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
        } else if (!(o.f == o.f)) {
            it.err = QE_DEVERR_NUMERIC;
        }
    }
    if (lane == 0) {
        f[b] = o.f;
        if (g) g[b] = o.g;
        if (delta) delta[b] = o.delta;
        if (it.err) atomicOr(a.err, it.err);
    }
}

// Marks circuits whose width is outside 1..6 (mixed-width batches only).
__global__ void width_check_kernel(BatchArgs a, float* f, float* g, float* delta) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const int n = a.nq[b];
    if (n >= 1 && n <= MAX_QUBITS) return;
    f[b] = __builtin_nanf("");
    if (g) g[b] = __builtin_nanf("");
    if (delta) delta[b] = __builtin_nanf("");
    atomicOr(a.err, (uint32_t)QE_DEVERR_WIDTH);
}

// LDS-staged path, W wavefronts per circuit (see run_lds_path).
template <int NQ, int W, bool FILTER, bool IDENT, bool ANG = false>
__global__ __launch_bounds__(64 * W) void lds32_kernel(BatchArgs a, float* __restrict__ f,
                                                       float* __restrict__ g,
                                                       float* __restrict__ delta,
                                                       float* __restrict__ U_out) {
    constexpr int N = 1 << NQ, CW = N / W;
    __shared__ float2 M[N * N];
    __shared__ uint4 GT[W][ANG ? GATE_TABLE_ANGLED : GATE_TABLE];
    const int b = blockIdx.x;
    const int lane = (int)lane_id(), wave = (int)(threadIdx.x >> 6);
    Item it = resolve(a, b, !IDENT);
    if (FILTER && it.n != NQ) return;
    if (it.err == 0 && it.n != NQ) it.err = QE_DEVERR_WIDTH;
    bool ok = it.err == 0;
    RowMap map{};
    if (ok) {
        const int L = it.L;
        auto src = [&](int ch) { return batch_gate<ANG>(it, ch * 64 + lane); };
        const float* T = IDENT ? nullptr : reinterpret_cast<const float*>(a.targets) + 2 * it.toff;
        ok = run_lds_path<NQ, W, IDENT>(M, GT[wave], T, L, src, IDENT ? nullptr : &map);
        if (!ok) it.err = QE_DEVERR_DESC;
    }
    if (IDENT) {
        __syncthreads();
        float2* U = reinterpret_cast<float2*>(U_out) + (size_t)N * N * b;
        const float nan = __builtin_nanf("");
        for (int e = threadIdx.x; e < N * N; e += 64 * W) U[e] = ok ? M[e] : make_float2(nan, nan);
        if (threadIdx.x == 0 && it.err) atomicOr(a.err, it.err);
        return;
    }
    // fitness, in the width's fixed order
    constexpr int WR = reduction_waves<NQ>();
    static_assert(WR == 1 || WR == W, "the reduction's wavefronts are the circuit's");
    __shared__ float red[4][3];
    if constexpr (W > 1) __syncthreads();      // every wavefront's columns are in place
    if (WR == 1 && wave != 0) return;
    float gv, dlt;
    const float fv = canonical_fitness<NQ, WR>(M, map, a.mode, &gv, &dlt, WR == 1 ? 0 : wave, red);
    if (wave == 0 && lane == 0) {
        const float nan = __builtin_nanf("");
        if (ok && !(fv == fv)) it.err = QE_DEVERR_NUMERIC;
        f[b] = ok ? fv : nan;
        if (g) g[b] = ok ? gv : nan;
        if (delta) delta[b] = ok ? dlt : nan;
        if (it.err) atomicOr(a.err, it.err);
    }
}

// ----------------------------------------------- mixed widths, one launch
// Circuits of a mixed-width batch are ordered by cost, widest first and,
// within a width, longest first (classes of 8 gates), by a one-workgroup
// counting sort; one launch then gives every workgroup (4 wavefronts) one
// work item: a circuit of width 6 (4 waves), two of width 5 (2 waves each),
// or four of width <= 4 (one wave each; LDS-staged for 4, one entry per lane
// below), so an item's circuits have similar lengths.  Workgroups are
// dispatched in index order, so the heaviest items start first
// (longest-processing-time order).
constexpr int MIX_BUCKETS = 7;          // widths 6..1, then malformed widths
constexpr int MIX_LCLASSES = 16;        // lengths >= 120, 112..119, ..., 8..15, < 8

__device__ __forceinline__ int mix_bucket(int n) { return (n >= 1 && n <= MAX_QUBITS) ? 6 - n : 6; }

// Sort key of circuit b: width bucket, then length class (longest first; a
// malformed range only lands in some class, the item reports it).
__device__ __forceinline__ int mix_key(const BatchArgs& a, int b) {
    const int64_t len = a.uniform_L > 0 ? (int64_t)a.uniform_L : (int64_t)a.goff[b + 1] - a.goff[b];
    const int lc = len >= 120 ? 0 : (len < 8 ? MIX_LCLASSES - 1 : MIX_LCLASSES - 1 - (int)(len >> 3));
    return mix_bucket(a.nq[b]) * MIX_LCLASSES + lc;
}
// circuits per work item: one of width 6 (four wavefronts), three of width
// 5 with one wavefront each (their 8 KB matrices and gate tables fill the
// 32 KB of LDS; the fourth wavefront idles) or two with two wavefronts each,
// four of the other widths
__device__ __forceinline__ int mix_per_item(int k, int w5) {
    return k == 0 ? 1 : (k == 1 ? (w5 == 2 ? 2 : 3) : 4);
}

// meta: [0..7) first order position, [8..15) first item (8 entries, the last
// the total), [16..23) count per bucket.
__global__ __launch_bounds__(1024) void mix_bucket_kernel(BatchArgs a, int32_t* order, int32_t* meta) {
    constexpr int K = MIX_BUCKETS * MIX_LCLASSES;
    __shared__ int cnt[K], cursor[K];
    const int tid = threadIdx.x;
    for (int k = tid; k < K; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    for (int b = tid; b < a.B; b += blockDim.x) atomicAdd(&cnt[mix_key(a, b)], 1);
    __syncthreads();
    static_assert(K <= 128, "two keys per lane of one wavefront");
    if (tid < 64) {
        // exclusive prefix sum of the K counts over one wavefront, two per lane
        const int k0 = 2 * tid;
        const int c0 = k0 < K ? cnt[k0] : 0, c1 = k0 + 1 < K ? cnt[k0 + 1] : 0;
        int incl = c0 + c1;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(incl, d, 64);
            if (tid >= d) incl += o;
        }
        const int excl = incl - c0 - c1;
        if (k0 < K) cursor[k0] = excl;
        if (k0 + 1 < K) cursor[k0 + 1] = excl + c0;
    }
    __syncthreads();
    if (tid == 0) {
        // per width: first order position, first item, count (every circuit
        // has a key, so the last width ends at B)
        int item = 0;
        for (int k = 0; k < MIX_BUCKETS; ++k) {
            const int pos = cursor[k * MIX_LCLASSES];
            const int end = k + 1 < MIX_BUCKETS ? cursor[(k + 1) * MIX_LCLASSES] : a.B;
            meta[k] = pos;
            meta[8 + k] = item;
            meta[16 + k] = end - pos;
            item += (end - pos + mix_per_item(k, a.mix_w5) - 1) / mix_per_item(k, a.mix_w5);
        }
        meta[8 + MIX_BUCKETS] = item;
    }
    __syncthreads();
    for (int b = tid; b < a.B; b += blockDim.x) order[atomicAdd(&cursor[mix_key(a, b)], 1)] = b;
}

template <int NQ, int W>
__device__ __forceinline__ void mix_lds_item(const BatchArgs& a, int b, float2* M, uint4* gt,
                                             float (*red)[3], float* f, float* g, float* delta) {
    const int lane = (int)lane_id(), wave = (int)(threadIdx.x >> 6);
    Item it;
    it.err = 1;
    if (b >= 0) it = resolve(a, b);
    bool ok = it.err == 0;
    RowMap map{};
    if (ok) {
        const uint16_t* gp = it.g;
        const int L = it.L;
        auto src = [&](int ch) -> uint32_t {
            const int p = ch * 64 + lane;
            return p < L ? (uint32_t)gp[p] : 0u;
        };
        const float* T = reinterpret_cast<const float*>(a.targets) + 2 * it.toff;
        ok = run_lds_path<NQ, W, false>(M, gt, T, L, src, &map, wave % W);
        if (!ok) it.err = QE_DEVERR_DESC;
    }
    constexpr int WR = reduction_waves<NQ>();
    static_assert(WR == 1 || WR == W, "the reduction's wavefronts are the circuit's");
    if constexpr (W > 1) __syncthreads();     // every wavefront's columns are in place
    if (WR == 1 && wave % W != 0) return;
    float gv, dv;
    const float fv = canonical_fitness<NQ, WR>(M, map, a.mode, &gv, &dv, WR == 1 ? 0 : wave % W, red);
    if (b >= 0 && wave % W == 0 && lane == 0) {
        const float nan = __builtin_nanf("");
        if (ok && !(fv == fv)) it.err = QE_DEVERR_NUMERIC;
        f[b] = ok ? fv : nan;
        if (g) g[b] = ok ? gv : nan;
        if (delta) delta[b] = ok ? dv : nan;
        if (it.err) atomicOr(a.err, it.err);
    }
}

template <int NQ>
__device__ __forceinline__ void mix_wave_item(const BatchArgs& a, int b, float* f, float* g,
                                              float* delta) {
    if (b < 0) return;
    const int lane = (int)lane_id();
    Item it = resolve(a, b);
    FitOut o{__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
    if (it.err == 0) {
        const uint16_t* gp = it.g;
        const int L = it.L;
        auto src = [&](int ch) -> uint32_t {
            const int p = ch * 64 + lane;
            return p < L ? (uint32_t)gp[p] : 0u;
        };
        const float* T = reinterpret_cast<const float*>(a.targets) + 2 * it.toff;
        if (!run_small_path<NQ, false>(T, L, src, nullptr, &o, a.mode)) {
            it.err = QE_DEVERR_DESC;
            o = FitOut{__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
        } else if (!(o.f == o.f)) {
            it.err = QE_DEVERR_NUMERIC;
        }
    }
    if (lane == 0) {
        f[b] = o.f;
        if (g) g[b] = o.g;
        if (delta) delta[b] = o.delta;
        if (it.err) atomicOr(a.err, it.err);
    }
}

__global__ __launch_bounds__(256) void mix_kernel(BatchArgs a, const int32_t* __restrict__ order,
                                                  const int32_t* __restrict__ meta,
                                                  float* __restrict__ f, float* __restrict__ g,
                                                  float* __restrict__ delta) {
    __shared__ float2 M[4096];
    __shared__ float red[4][3];
    const int item = blockIdx.x;
    if (item >= meta[8 + MIX_BUCKETS]) return;
    int k = 0;
    while (k + 1 < MIX_BUCKETS && item >= meta[8 + k + 1]) ++k;
    const int wave = (int)(threadIdx.x >> 6);
    const int per = mix_per_item(k, a.mix_w5);
    const int local = (item - meta[8 + k]) * per;
    const int sub = per == 1 ? 0 : (per == 2 ? wave >> 1 : wave);
    int b = sub < per && local + sub < meta[16 + k] ? order[meta[k] + local + sub] : -1;
    if (b >= a.B) b = -1;        // an order written for another batch never indexes past this one
    switch (k) {
        // (widths 4 and 5 run one circuit per wavefront, each with its gate table)
        case 0: mix_lds_item<6, 4>(a, b, M, nullptr, red, f, g, delta); break;
        case 1:
            if (a.mix_w5 == 2) mix_lds_item<5, 2>(a, b, M + sub * 1024, nullptr, red, f, g, delta);
            else if (wave < 3)   // gate tables in the last quarter of M
                mix_lds_item<5, 1>(a, b, M + sub * 1024, reinterpret_cast<uint4*>(M + 3072) + wave * GATE_TABLE,
                                   red, f, g, delta);
            break;
        case 2:   // gate tables after the four 16 x 16 matrices
            mix_lds_item<4, 1>(a, b, M + sub * 256, reinterpret_cast<uint4*>(M + 1024) + wave * GATE_TABLE, red,
                               f, g, delta);
            break;
        case 3: mix_wave_item<3>(a, b, f, g, delta); break;
        case 4: mix_wave_item<2>(a, b, f, g, delta); break;
        case 5: mix_wave_item<1>(a, b, f, g, delta); break;
        default:
            if (b >= 0 && lane_id() == 0) {
                const float nan = __builtin_nanf("");
                f[b] = nan;
                if (g) g[b] = nan;
                if (delta) delta[b] = nan;
                atomicOr(a.err, (uint32_t)QE_DEVERR_WIDTH);
            }
            break;
    }
}

// --------------------------------------------------------- generic LDS path
template <typename Real, bool IDENT>
__global__ __launch_bounds__(256) void lds_kernel(BatchArgs a, Real* __restrict__ f,
                                                  Real* __restrict__ g, Real* __restrict__ delta,
                                                  Real* __restrict__ U_out) {
    const int b = blockIdx.x;
    Item it = resolve(a, b, !IDENT);
    const Real* T = (IDENT || it.err) ? nullptr : reinterpret_cast<const Real*>(a.targets) + 2 * it.toff;
    Real* U = nullptr;
    if (IDENT) U = U_out + (size_t)2 * ((size_t)1 << (2 * a.uniform_n)) * b;
    // dynamic LDS: two planes of 4^n reals for the batch's (largest) width
    Real* Mr = generic_lds<Real>();
    Real* Mi = Mr + ((size_t)1 << (2 * (a.uniform_n > 0 ? a.uniform_n : MAX_QUBITS)));
    lds_generic_body<Real, IDENT>(it.n, it.L, it.g, it.ang, T, it.err, f + (f ? b : 0),
                                  g ? g + b : nullptr, delta ? delta + b : nullptr, U, a.err, a.mode,
                                  Mr, Mi);
}

// LDS bytes of lds_kernel for a batch
static size_t lds_kernel_bytes(const BatchArgs& a, size_t real_bytes) {
    return generic_lds_bytes(a.uniform_n > 0 ? a.uniform_n : MAX_QUBITS, real_bytes);
}

// ------------------------------------------------------------------ launchers
// Per-width schedule: which kernel evaluates a circuit of width n on the
// FP32 path.  path: QE_PATH_FP32 (default schedule), QE_PATH_FP32_REG,
// QE_PATH_FP32_LDS.
static bool use_lds(int n, int path, int L) {
    if (n <= 3) return false;
    if (path == QE_PATH_FP32_REG) return false;
    if (path == QE_PATH_FP32_LDS) return true;
    return schedule_for(n, L).lds != 0;
}

// length of the batch's circuits for the schedule (uneven batches: the long class)
static int sched_len(const BatchArgs& a) { return a.uniform_L > 0 ? a.uniform_L : 32; }

// Angled batches (ANG): the one-element-per-lane kernel for n <= 3 and the
// LDS-staged one above (the register-resident path has no Ising kinds).
template <bool FILTER, bool ANG = false>
static void launch_width(const BatchArgs& a, int n, bool lds, float* f, float* g, float* delta,
                         hipStream_t s) {
    const dim3 wgrid((a.B + WPB - 1) / WPB), wblock(64 * WPB);
    if constexpr (ANG) {
        switch (n) {
            case 1: wave_kernel<1, FILTER, true><<<wgrid, wblock, 0, s>>>(a, f, g, delta); break;
            case 2: wave_kernel<2, FILTER, true><<<wgrid, wblock, 0, s>>>(a, f, g, delta); break;
            case 3: wave_kernel<3, FILTER, true><<<wgrid, wblock, 0, s>>>(a, f, g, delta); break;
            case 4: lds32_kernel<4, 1, FILTER, false, true><<<a.B, 64, 0, s>>>(a, f, g, delta, nullptr); break;
            case 5:
                if (schedule_for(5, sched_len(a), SCHED_ISING).waves == 2)
                    lds32_kernel<5, 2, FILTER, false, true><<<a.B, 128, 0, s>>>(a, f, g, delta, nullptr);
                else
                    lds32_kernel<5, 1, FILTER, false, true><<<a.B, 64, 0, s>>>(a, f, g, delta, nullptr);
                break;
            default: lds32_kernel<6, 4, FILTER, false, true><<<a.B, 256, 0, s>>>(a, f, g, delta, nullptr); break;
        }
        return;
    }
    if (lds) {
        switch (n) {
            case 4: lds32_kernel<4, 1, FILTER, false><<<a.B, 64, 0, s>>>(a, f, g, delta, nullptr); break;
            case 5:
                if (schedule_for(5, sched_len(a)).waves == 2)
                    lds32_kernel<5, 2, FILTER, false><<<a.B, 128, 0, s>>>(a, f, g, delta, nullptr);
                else
                    lds32_kernel<5, 1, FILTER, false><<<a.B, 64, 0, s>>>(a, f, g, delta, nullptr);
                break;
            default: lds32_kernel<6, 4, FILTER, false><<<a.B, 256, 0, s>>>(a, f, g, delta, nullptr); break;
        }
        return;
    }
    switch (n) {
        case 1: wave_kernel<1, FILTER><<<wgrid, wblock, 0, s>>>(a, f, g, delta); break;
        case 2: wave_kernel<2, FILTER><<<wgrid, wblock, 0, s>>>(a, f, g, delta); break;
        case 3: wave_kernel<3, FILTER><<<wgrid, wblock, 0, s>>>(a, f, g, delta); break;
        case 4: wave_kernel<4, FILTER><<<wgrid, wblock, 0, s>>>(a, f, g, delta); break;
        case 5: wave_kernel<5, FILTER><<<wgrid, wblock, 0, s>>>(a, f, g, delta); break;
        default: wave_kernel<6, FILTER><<<wgrid, wblock, 0, s>>>(a, f, g, delta); break;
    }
}

hipError_t launch_eval_fp32(const BatchArgs& a, int path, float* f, float* g, float* delta,
                            int32_t* work, hipStream_t s) {
    if (a.B == 0) return hipSuccess;
    if (a.angles) {
        if (a.uniform_n > 0) {
            launch_width<false, true>(a, a.uniform_n, true, f, g, delta, s);
        } else {
            width_check_kernel<<<(a.B + 255) / 256, 256, 0, s>>>(a, f, g, delta);
            for (int n = 1; n <= MAX_QUBITS; ++n) launch_width<true, true>(a, n, true, f, g, delta, s);
        }
    } else if (a.uniform_n > 0) {
        launch_width<false>(a, a.uniform_n, use_lds(a.uniform_n, path, sched_len(a)), f, g, delta, s);
    } else if (path == QE_PATH_FP32 && work) {
        // one launch over width-sorted work items (LDS-staged for n >= 4)
        mix_bucket_kernel<<<1, 1024, 0, s>>>(a, work + MIX_WORK_META, work);
        mix_kernel<<<a.B, 256, 0, s>>>(a, work + MIX_WORK_META, work, f, g, delta);
    } else {
        width_check_kernel<<<(a.B + 255) / 256, 256, 0, s>>>(a, f, g, delta);
        for (int n = 1; n <= MAX_QUBITS; ++n)
            launch_width<true>(a, n, use_lds(n, path, sched_len(a)), f, g, delta, s);
    }
    return hipGetLastError();
}

// The phase-insensitive fitness is sum |U_ij|^2 |T_ij|^2 / 2^n; the kernels
// evaluate it as the diagonal overlap of U T^dagger, which equals it exactly
// when every entry of T has modulus 0 or 1.  One wavefront per circuit (one in
// all for a shared target) checks the target; a circuit whose target has an
// entry of modulus strictly between gets NaN and QE_DEVERR_TARGET.  Runs
// after the evaluation, whose outputs it overwrites.
template <typename Real>
__global__ void target_check_kernel(BatchArgs a, Real* f, Real* g, Real* delta) {
    const int lane = (int)lane_id();
    const bool shared = a.tstride == 0 && a.uniform_n > 0;
    const int b = shared ? 0 : (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (b >= a.B || (shared && (blockIdx.x > 0 || threadIdx.x >= 64))) return;
    const Item it = resolve(a, b, true);
    if (it.err) return;                    // malformed circuits report already
    const int NN = 1 << (2 * it.n);
    const Real* T = reinterpret_cast<const Real*>(a.targets) + 2 * it.toff;
    const Real tol = sizeof(Real) == 8 ? (Real)1e-9 : (Real)1e-5;
    bool bad = false;
    for (int e = lane; e < NN; e += 64) {
        const Real x = T[2 * e], y = T[2 * e + 1];
        const Real m = x * x + y * y;
        if (!(m <= tol || (m - (Real)1 <= tol && (Real)1 - m <= tol))) bad = true;
    }
    if (__ballot(bad) == 0ull) return;
    const Real nan = (Real)__builtin_nan("");
    auto mark = [&](int c) {
        f[c] = nan;
        if (g) g[c] = nan;
        if (delta) delta[c] = nan;
    };
    if (shared) {
        for (int c = lane; c < a.B; c += 64) mark(c);
    } else if (lane == 0) {
        mark(b);
    }
    if (lane == 0) atomicOr(a.err, (uint32_t)QE_DEVERR_TARGET);
}

hipError_t launch_target_check(const BatchArgs& a, bool fp64, void* f, void* g, void* delta,
                               hipStream_t s) {
    if (a.B == 0 || a.mode != QE_FIT_PHASE_INSENSITIVE) return hipSuccess;
    const unsigned grid = (a.tstride == 0 && a.uniform_n > 0) ? 1u : (unsigned)((a.B + 3) / 4);
    if (fp64) target_check_kernel<double><<<grid, 256, 0, s>>>(a, (double*)f, (double*)g, (double*)delta);
    else target_check_kernel<float><<<grid, 256, 0, s>>>(a, (float*)f, (float*)g, (float*)delta);
    return hipGetLastError();
}

hipError_t launch_mix_sort(const BatchArgs& a, int32_t* work, hipStream_t s) {
    if (a.B > 0) mix_bucket_kernel<<<1, 1024, 0, s>>>(a, work + MIX_WORK_META, work);
    return hipGetLastError();
}

hipError_t launch_mix_eval(const BatchArgs& a, const int32_t* work, float* f, float* g, float* delta,
                           hipStream_t s) {
    if (a.B > 0) mix_kernel<<<a.B, 256, 0, s>>>(a, work + MIX_WORK_META, work, f, g, delta);
    return hipGetLastError();
}

hipError_t launch_eval_lds(const BatchArgs& a, bool fp64, void* f, void* g, void* delta,
                           hipStream_t s) {
    if (a.B == 0) return hipSuccess;
    if (fp64)
        lds_kernel<double, false><<<a.B, 256, lds_kernel_bytes(a, 8), s>>>(a, (double*)f, (double*)g,
                                                                           (double*)delta, nullptr);
    else
        lds_kernel<float, false><<<a.B, 256, lds_kernel_bytes(a, 4), s>>>(a, (float*)f, (float*)g,
                                                                          (float*)delta, nullptr);
    return hipGetLastError();
}

hipError_t launch_unitary(const BatchArgs& a, bool fp64, void* out, hipStream_t s) {
    if (a.B == 0) return hipSuccess;
    if (fp64) {
        lds_kernel<double, true><<<a.B, 256, lds_kernel_bytes(a, 8), s>>>(a, nullptr, nullptr, nullptr,
                                                                          (double*)out);
    } else {
        float* o = (float*)out;
        switch (a.uniform_n) {
            case 1: lds_kernel<float, true><<<a.B, 256, lds_kernel_bytes(a, 4), s>>>(a, nullptr, nullptr, nullptr, o); break;
            case 2: lds_kernel<float, true><<<a.B, 256, lds_kernel_bytes(a, 4), s>>>(a, nullptr, nullptr, nullptr, o); break;
            case 3: lds_kernel<float, true><<<a.B, 256, lds_kernel_bytes(a, 4), s>>>(a, nullptr, nullptr, nullptr, o); break;
            case 4:
                if (a.angles) lds32_kernel<4, 1, false, true, true><<<a.B, 64, 0, s>>>(a, nullptr, nullptr, nullptr, o);
                else lds32_kernel<4, 1, false, true><<<a.B, 64, 0, s>>>(a, nullptr, nullptr, nullptr, o);
                break;
            case 5:
                if (a.angles) lds32_kernel<5, 1, false, true, true><<<a.B, 64, 0, s>>>(a, nullptr, nullptr, nullptr, o);
                else lds32_kernel<5, 1, false, true><<<a.B, 64, 0, s>>>(a, nullptr, nullptr, nullptr, o);
                break;
            default:
                if (a.angles) lds32_kernel<6, 4, false, true, true><<<a.B, 256, 0, s>>>(a, nullptr, nullptr, nullptr, o);
                else lds32_kernel<6, 4, false, true><<<a.B, 256, 0, s>>>(a, nullptr, nullptr, nullptr, o);
                break;
        }
    }
    return hipGetLastError();
}

}  // namespace qe
