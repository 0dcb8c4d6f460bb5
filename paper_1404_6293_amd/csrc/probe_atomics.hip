// probe_atomics.hip -- throughput probes that give the atomic rooflines of
// the raster pipeline their denominators on the GPU at hand (a measurement
// tool built beside libpk, not part of the pipeline; include/pk_probe.h).
//
//   pkp_lds_min_u64     64-bit LDS atomic min into a per-workgroup tile of
//                       B*B keys at addresses uniform over the tile (the
//                       fragments of many triangles landing in one bin's
//                       depth tile), with or without the returned old value
//   pkp_global_min_u64  one device-scope 64-bit atomic min per entry of an
//                       address list (e.g. the pixels of an unbinned frame's
//                       fragments, in submission order)
//   pkp_global_add_f32  one device-scope float32 atomic add per entry of an
//                       address list (e.g. the scatters of the backward pass)
//
// Every probe is a plain, bounded grid: no persistent loop, no waits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pk_probe.h"

namespace {

constexpr int kThreads = 256;

__device__ inline uint32_t xorshift(uint32_t &s) {
    s ^= s << 13;
    s ^= s >> 17;
    s ^= s << 5;
    return s;
}

template <int TILE, bool RTN>
__global__ __launch_bounds__(kThreads) void k_lds_min(int iters, unsigned long long *sink) {
    __shared__ unsigned long long tile[TILE];
    for (int i = threadIdx.x; i < TILE; i += kThreads) tile[i] = ~0ull;
    __syncthreads();
    uint32_t s = 0x9e3779b9u ^ (blockIdx.x * kThreads + threadIdx.x) * 0x85ebca6bu;
    if (s == 0) s = 1;
    unsigned long long acc = 0;
    for (int k = 0; k < iters; ++k) {
        const uint32_t r = xorshift(s);
        const unsigned long long key = ((unsigned long long)(r >> 8) << 32) | (uint32_t)k;
        if (RTN)
            acc += atomicMin(&tile[r % TILE], key);
        else
            atomicMin(&tile[r % TILE], key);
    }
    __syncthreads();
    // one value per workgroup keeps the tile (and the returned values) live
    if (threadIdx.x == 0) sink[blockIdx.x] = tile[0] + acc;
    else if (RTN && acc == 0x5eed5eed5eedull) sink[blockIdx.x] = acc;   // (never)
}

__global__ __launch_bounds__(kThreads) void k_global_min(unsigned long long *keys,
                                                         const int32_t *addr, int64_t m) {
    const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i >= m) return;
    // distinct keys that keep changing the minimum now and then
    const unsigned long long key = ((unsigned long long)((uint32_t)i * 2654435761u) << 32) |
                                   (uint32_t)i;
    atomicMin(keys + addr[i], key);
}

__global__ __launch_bounds__(kThreads) void k_global_add(float *dst, const int32_t *addr,
                                                         const float *vals, int64_t m) {
    const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i >= m) return;
    atomicAdd(dst + addr[i], vals ? vals[i] : 1.0f);
}

int status(hipError_t e) { return e == hipSuccess ? 0 : 3; }

}  // namespace

extern "C" {

int pkp_lds_min_u64(int tile_keys, int with_return, int workgroups, int iters,
                    unsigned long long *sink, void *stream) {
    if (workgroups < 1 || iters < 1 || !sink) return 1;
    const hipStream_t st = (hipStream_t)stream;
    const dim3 g((unsigned)workgroups), b(kThreads);
#define PKP_LDS(T)                                                                      \
    case T:                                                                             \
        if (with_return)                                                                \
            hipLaunchKernelGGL((k_lds_min<T, true>), g, b, 0, st, iters, sink);         \
        else                                                                            \
            hipLaunchKernelGGL((k_lds_min<T, false>), g, b, 0, st, iters, sink);        \
        break;
    switch (tile_keys) {
        PKP_LDS(64)
        PKP_LDS(256)
        PKP_LDS(1024)
        PKP_LDS(4096)
    default:
        return 1;
    }
#undef PKP_LDS
    return status(hipGetLastError());
}

int pkp_global_min_u64(unsigned long long *keys, const int32_t *addr, int64_t m, void *stream) {
    if (m < 0 || (m > 0 && (!keys || !addr))) return 1;
    if (m == 0) return 0;
    hipLaunchKernelGGL(k_global_min, dim3((unsigned)((m + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, (hipStream_t)stream, keys, addr, m);
    return status(hipGetLastError());
}

int pkp_global_add_f32(float *dst, const int32_t *addr, const float *vals, int64_t m,
                       void *stream) {
    if (m < 0 || (m > 0 && (!dst || !addr))) return 1;
    if (m == 0) return 0;
    hipLaunchKernelGGL(k_global_add, dim3((unsigned)((m + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, (hipStream_t)stream, dst, addr, vals, m);
    return status(hipGetLastError());
}

}  // extern "C"
