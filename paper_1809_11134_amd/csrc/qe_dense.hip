// The paper's own evaluation scheme (Sec. IV-C, steps 3-5), kept as an
// ablation of the per-gate row updates: every gate of a circuit is expanded to
// its full 2^n x 2^n segment matrix -- the Kronecker product of its 2 x 2
// factor on its wire with identities on the other wires; a controlled gate as
// the sum of the products with the projectors |0><0| and |1><1| on the control
// wire; the interaction J as its +-1 template diagonal exponentiated element
// by element -- and the circuit is the product of the segment matrices,
// applied to T^dagger.  Each gate costs N^3 complex multiply-adds here
// instead of the N^2 (or fewer) entry updates of the per-gate path.
//
// One workgroup of 256 threads per circuit; M, the segment matrix G and the
// product live in LDS (6 x N^2 floats); each thread owns a TD x TD tile of the
// product (TD = N / 16 for n >= 4, so that the 256 tiles cover it).
#include "../../include/qe.h"
#include "qe_eval_core.hpp"
#include "qe_internal.hpp"

namespace qe {

template <typename Real>
__device__ __forceinline__ Cplx<Real> cmul(Cplx<Real> a, Cplx<Real> b) {
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}

// Entry (r, k) of the expanded segment matrix of gate d (kind, wires) whose
// 2 x 2 factor is U (rotations and discrete kinds; in LDS as re, im of
// [[u0, u1], [u2, u3]], so that picking an entry is an indexed LDS read) or
// whose half-angle cosine and sine are c, s (the interaction).
template <int NQ>
__device__ __forceinline__ Cplx<float> segment_entry(int kind, int t, int ctl_w, const float* U,
                                                     float c, float s, int r, int k) {
    const Cplx<float> one = {1.0f, 0.0f}, zero = {0.0f, 0.0f};
    if (kind == KIND_ZZ) {
        if (r != k) return zero;
        const int odd = ((r >> (NQ - 1 - t)) ^ (r >> (NQ - 1 - ctl_w))) & 1;
        return {c, odd ? s : -s};          // exp(-i theta/2 * (+-1))
    }
    const bool ctl = kind_controlled(kind);
    Cplx<float> p_on = one, p_off = one;   // the two Kronecker products
#pragma unroll
    for (int w = 0; w < NQ; ++w) {
        const int rb = (r >> (NQ - 1 - w)) & 1, kb = (k >> (NQ - 1 - w)) & 1;
        const Cplx<float> id = rb == kb ? one : zero;
        if (w == t) {
            const Cplx<float> u = {U[4 * rb + 2 * kb], U[4 * rb + 2 * kb + 1]};
            p_on = cmul(p_on, u);
            p_off = cmul(p_off, id);
        } else if (ctl && w == ctl_w) {
            p_on = cmul(p_on, (rb & kb) ? one : zero);        // |1><1|
            p_off = cmul(p_off, (!rb && !kb) ? one : zero);   // |0><0|
        } else {
            p_on = cmul(p_on, id);
            p_off = cmul(p_off, id);
        }
    }
    return ctl ? Cplx<float>{p_on.r + p_off.r, p_on.i + p_off.i} : p_on;
}

template <int NQ, bool FILTER, bool ANG>
__global__ __launch_bounds__(256) void dense_kernel(BatchArgs a, float* __restrict__ f,
                                                    float* __restrict__ g, float* __restrict__ delta) {
    constexpr int N = 1 << NQ, NN = N * N;
    constexpr int TD = N >= 16 ? N / 16 : 1, NT = N / TD;   // tile edge, tiles per edge
    __shared__ float Mr[NN], Mi[NN], Gr[NN], Gi[NN], Pr[NN], Pi[NN];
    __shared__ float red[8];
    __shared__ float Uf[8];
    const int b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    Item it = resolve_item(a, b, true);
    if (FILTER && it.n != NQ) return;
    if (it.err == 0 && it.n != NQ) it.err = QE_DEVERR_WIDTH;
    bool ok = it.err == 0;
    if (ok) {
        const float* T = reinterpret_cast<const float*>(a.targets) + 2 * it.toff;
        for (int e = tid; e < NN; e += nt) {       // M_0 = T^dagger
            const int i = e / N, j = e % N;
            Mr[e] = T[2 * (j * N + i)];
            Mi[e] = -T[2 * (j * N + i) + 1];
        }
        __syncthreads();
        for (int l = 0; l < it.L; ++l) {
            const uint32_t d = it.g[l];
            if (!desc_valid<ANG>(d, NQ)) { ok = false; break; }
            const int kind = d & 15;
            if (kind == KIND_I) continue;
            const int t = (d >> 4) & 15, cw = (d >> 8) & 15;
            float c = 1.0f, s = 0.0f;
            Cplx<float> Ua[4] = {{1.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}, {1.0f, 0.0f}};
            if constexpr (ANG) {
                if (kind_ising(kind)) half_angle(it.ang[l], &c, &s);
            }
            if (kind >= KIND_RX && kind <= KIND_RZ) rotation_coeffs<float>(kind, c, s, Ua);
            else if (kind != KIND_ZZ) gate_coeffs<float>(kind, Ua);
            if (tid == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) { Uf[2 * q] = Ua[q].r; Uf[2 * q + 1] = Ua[q].i; }
            }
            __syncthreads();
            // steps 3-4: the segment matrix
            for (int e = tid; e < NN; e += nt) {
                const Cplx<float> v = segment_entry<NQ>(kind, t, cw, Uf, c, s, e / N, e % N);
                Gr[e] = v.r;
                Gi[e] = v.i;
            }
            __syncthreads();
            // step 5: P = G M, one TD x TD tile per thread
            if (tid < NT * NT) {
                const int r0 = (tid / NT) * TD, c0 = (tid % NT) * TD;
                float ar[TD][TD], ai[TD][TD];
#pragma unroll
                for (int x = 0; x < TD; ++x)
#pragma unroll
                    for (int y = 0; y < TD; ++y) ar[x][y] = ai[x][y] = 0.0f;
                for (int k = 0; k < N; ++k) {
                    float gr[TD], gi[TD], mr[TD], mi[TD];
#pragma unroll
                    for (int x = 0; x < TD; ++x) { gr[x] = Gr[(r0 + x) * N + k]; gi[x] = Gi[(r0 + x) * N + k]; }
#pragma unroll
                    for (int y = 0; y < TD; ++y) { mr[y] = Mr[k * N + c0 + y]; mi[y] = Mi[k * N + c0 + y]; }
#pragma unroll
                    for (int x = 0; x < TD; ++x)
#pragma unroll
                        for (int y = 0; y < TD; ++y) {
                            ar[x][y] += gr[x] * mr[y] - gi[x] * mi[y];
                            ai[x][y] += gr[x] * mi[y] + gi[x] * mr[y];
                        }
                }
#pragma unroll
                for (int x = 0; x < TD; ++x)
#pragma unroll
                    for (int y = 0; y < TD; ++y) {
                        Pr[(r0 + x) * N + c0 + y] = ar[x][y];
                        Pi[(r0 + x) * N + c0 + y] = ai[x][y];
                    }
            }
            __syncthreads();
            for (int e = tid; e < NN; e += nt) { Mr[e] = Pr[e]; Mi[e] = Pi[e]; }
            __syncthreads();
        }
        if (!ok) it.err = QE_DEVERR_DESC;
    }
    lds_fitness<float>(Mr, Mi, N, ok, it.err, f + b, g ? g + b : nullptr, delta ? delta + b : nullptr,
                       a.err, a.mode, red);
}

template <bool FILTER, bool ANG>
static void launch_dense_width(const BatchArgs& a, int n, float* f, float* g, float* delta, hipStream_t s) {
    switch (n) {
        case 1: dense_kernel<1, FILTER, ANG><<<a.B, 256, 0, s>>>(a, f, g, delta); break;
        case 2: dense_kernel<2, FILTER, ANG><<<a.B, 256, 0, s>>>(a, f, g, delta); break;
        case 3: dense_kernel<3, FILTER, ANG><<<a.B, 256, 0, s>>>(a, f, g, delta); break;
        case 4: dense_kernel<4, FILTER, ANG><<<a.B, 256, 0, s>>>(a, f, g, delta); break;
        case 5: dense_kernel<5, FILTER, ANG><<<a.B, 256, 0, s>>>(a, f, g, delta); break;
        default: dense_kernel<6, FILTER, ANG><<<a.B, 256, 0, s>>>(a, f, g, delta); break;
    }
}

// Marks circuits whose width is outside 1..6 (mixed-width batches).
__global__ void dense_width_check_kernel(BatchArgs a, float* f, float* g, float* delta) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const int n = a.nq[b];
    if (n >= 1 && n <= MAX_QUBITS) return;
    f[b] = __builtin_nanf("");
    if (g) g[b] = __builtin_nanf("");
    if (delta) delta[b] = __builtin_nanf("");
    atomicOr(a.err, (uint32_t)QE_DEVERR_WIDTH);
}

hipError_t launch_eval_dense(const BatchArgs& a, float* f, float* g, float* delta, hipStream_t s) {
    if (a.B == 0) return hipSuccess;
    const bool ang = a.angles != nullptr;
    if (a.uniform_n > 0) {
        if (ang) launch_dense_width<false, true>(a, a.uniform_n, f, g, delta, s);
        else launch_dense_width<false, false>(a, a.uniform_n, f, g, delta, s);
    } else {
        dense_width_check_kernel<<<(a.B + 255) / 256, 256, 0, s>>>(a, f, g, delta);
        for (int n = 1; n <= MAX_QUBITS; ++n) {
            if (ang) launch_dense_width<true, true>(a, n, f, g, delta, s);
            else launch_dense_width<true, false>(a, n, f, g, delta, s);
        }
    }
    return hipGetLastError();
}

}  // namespace qe
