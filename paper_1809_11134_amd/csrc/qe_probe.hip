// Measurement helper: the LDS bandwidth the chip sustains, the denominator of
// the LDS rooflines of the per-gate kernels.  Not part of the method.
//
// Each workgroup of 256 threads owns 32 KB of LDS (2048 16-byte words, so
// five workgroups fit a compute unit's 160 KB).  Every wavefront instruction
// moves 64 consecutive 16-byte words (ds_read_b128 / ds_write_b128, one
// kilobyte, no bank conflicts); eight independent accesses are in flight per
// thread.  Mode 0 reads, mode 1 writes, mode 2 reads a word and writes it to
// another place (a copy inside LDS, counted as read plus write bytes).
#include <hip/hip_runtime.h>

#include "../../include/qe.h"

namespace {

constexpr int PROBE_BLOCK = 256;
constexpr int PROBE_WORDS = 2048;     // 32 KB of LDS per workgroup
constexpr int PROBE_UNROLL = 8;

template <int MODE>
__global__ __launch_bounds__(PROBE_BLOCK) void lds_probe_kernel(int iters, uint32_t salt,
                                                                uint32_t* __restrict__ sink) {
    __shared__ uint4 buf[PROBE_WORDS];
    const uint32_t t = threadIdx.x;
    for (uint32_t w = t; w < PROBE_WORDS; w += PROBE_BLOCK)
        buf[w] = make_uint4(w ^ salt, w + salt, w * 3u, w ^ 0x5a5a5a5au);
    __syncthreads();
    uint4 acc[PROBE_UNROLL];
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; ++u) acc[u] = make_uint4(t, u, salt, 0u);
    // word index of access u in iteration i: a whole kilobyte per wavefront,
    // the wavefront's kilobyte moving through the buffer (salt is 0 at run
    // time but unknown to the compiler, which must issue every access)
    uint32_t base = (t + salt) & (PROBE_WORDS - 1);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) {
            const uint32_t w = (base + (uint32_t)u * PROBE_BLOCK) & (PROBE_WORDS - 1);
            if (MODE == 0) {
                const uint4 v = buf[w];
                acc[u].x ^= v.x; acc[u].y += v.y; acc[u].z ^= v.z; acc[u].w += v.w;
            } else if (MODE == 1) {
                buf[w] = acc[u];
                acc[u].x += 1u;
            } else {
                acc[u] = buf[w];          // all eight reads are issued before the writes
            }
        }
        if (MODE == 2) {
#pragma unroll
            for (int u = 0; u < PROBE_UNROLL; ++u) {
                const uint32_t w = (base + (uint32_t)u * PROBE_BLOCK) & (PROBE_WORDS - 1);
                buf[w ^ 64u] = make_uint4(acc[u].x + 1u, acc[u].y, acc[u].z, acc[u].w);
            }
        }
        base = (base + 64u * PROBE_UNROLL + salt) & (PROBE_WORDS - 1);
    }
    __syncthreads();
    uint32_t r = 0;
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; ++u) r ^= acc[u].x ^ acc[u].y ^ acc[u].z ^ acc[u].w;
    r ^= buf[t].x;
    sink[blockIdx.x * PROBE_BLOCK + t] = r;
}

}  // namespace

extern "C" qe_status qe_probe_lds(int32_t mode, int32_t workgroups, int32_t iters, uint32_t* sink_dev,
                                  double* bytes_host, void* stream) {
    if (mode < 0 || mode > 2 || workgroups < 1 || iters < 1 || !sink_dev)
        return QE_ERR_INVALID;
    const hipStream_t s = (hipStream_t)stream;
    if (mode == 0) lds_probe_kernel<0><<<workgroups, PROBE_BLOCK, 0, s>>>(iters, 0u, sink_dev);
    else if (mode == 1) lds_probe_kernel<1><<<workgroups, PROBE_BLOCK, 0, s>>>(iters, 0u, sink_dev);
    else lds_probe_kernel<2><<<workgroups, PROBE_BLOCK, 0, s>>>(iters, 0u, sink_dev);
    if (hipGetLastError() != hipSuccess) return QE_ERR_DEVICE;
    if (bytes_host)
        *bytes_host = (double)workgroups * PROBE_BLOCK * iters * PROBE_UNROLL * 16.0 * (mode == 2 ? 2.0 : 1.0);
    return QE_OK;
}
