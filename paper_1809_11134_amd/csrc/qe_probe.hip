// Measurement helpers: the LDS bandwidth the chip sustains, the denominator of
// the LDS rooflines of the per-gate kernels, and the rate of random 16-byte
// record accesses in HBM, the floor of the QEQEA update.  Not part of the
// method.
//
// LDS probe:
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

// Random record probe: thread t takes record h(t) mod count of a buffer of
// 16-byte records (h: a multiply-xorshift hash of t and the salt, uniform
// over the buffer), reads it, and (MODE 1) writes it back changed -- the
// access pattern of a slot record in the update, one 128-byte line per
// record.
__device__ __forceinline__ uint32_t probe_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

template <int MODE>
__global__ __launch_bounds__(256) void record_probe_kernel(uint4* __restrict__ rec, uint32_t count,
                                                           uint32_t n, uint32_t salt,
                                                           uint32_t* __restrict__ sink) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t i = (uint32_t)(((uint64_t)probe_hash(t * 0x9E3779B9u + salt) * count) >> 32);
    uint4 v = rec[i];
    if (MODE == 1) {
        v.w = 0u;
        v.z += 1u;
        rec[i] = v;
    } else if (v.x == 0xFFFFFFFFu && v.y == salt) {
        sink[0] = v.z ^ v.w;          // (never true for the buffers the caller passes)
    }
}

}  // namespace

extern "C" qe_status qe_probe_records(int32_t mode, void* records_dev, int64_t count, int64_t accesses,
                                      uint32_t salt, uint32_t* sink_dev, void* stream) {
    if (mode < 0 || mode > 1 || !records_dev || !sink_dev || count < 1 || count > 0xFFFFFFFFll ||
        accesses < 0 || accesses > 0xFFFFFFFFll)
        return QE_ERR_INVALID;
    if (accesses == 0) return QE_OK;
    const hipStream_t s = (hipStream_t)stream;
    const uint32_t n = (uint32_t)accesses, blocks = (uint32_t)((accesses + 255) / 256);
    uint4* rec = static_cast<uint4*>(records_dev);
    if (mode == 0) record_probe_kernel<0><<<blocks, 256, 0, s>>>(rec, (uint32_t)count, n, salt, sink_dev);
    else record_probe_kernel<1><<<blocks, 256, 0, s>>>(rec, (uint32_t)count, n, salt, sink_dev);
    return hipGetLastError() == hipSuccess ? QE_OK : QE_ERR_DEVICE;
}

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
