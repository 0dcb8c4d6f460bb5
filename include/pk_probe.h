/*
 * pk_probe.h -- throughput probes of the hardware atomics the raster
 * pipeline relies on (libpk_probe.so, built beside libpk.so).  They measure
 * the denominators of the pipeline's atomic rooflines on the GPU at hand:
 * the 64-bit LDS atomic min of the per-bin depth test, the device-scope
 * 64-bit atomic min of the unbinned (whole-screen bin) depth test, and the
 * device-scope float32 atomic add of the backward pass.  Not part of the
 * rendering ABI (include/pk.h).
 *
 * Every pointer is a DEVICE pointer; `stream` is a hipStream_t (NULL = the
 * default stream).  The calls only enqueue one bounded kernel each; the
 * caller times them (e.g. with events around the call).  Return 0 on
 * success, 1 for an invalid argument (nothing enqueued), 3 when the launch
 * failed.
 */
#ifndef PK_PROBE_H
#define PK_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* `workgroups` workgroups of 256 threads; each thread issues `iters` 64-bit
 * atomic mins into its workgroup's LDS tile of `tile_keys` keys (64, 256,
 * 1024 or 4096: 8x8 to 64x64-pixel bins), at addresses drawn uniformly over
 * the tile by a per-thread xorshift generator.  with_return != 0 uses the
 * returned old value (the returning form of the instruction).  Operations =
 * workgroups * 256 * iters.  sink [workgroups] receives one value per
 * workgroup. */
int pkp_lds_min_u64(int tile_keys, int with_return, int workgroups, int iters,
                    unsigned long long *sink, void *stream);

/* For i in [0, m): atomicMin(&keys[addr[i]], key_i) with distinct keys. */
int pkp_global_min_u64(unsigned long long *keys, const int32_t *addr, int64_t m, void *stream);

/* For i in [0, m): atomicAdd(&dst[addr[i]], vals ? vals[i] : 1.0f). */
int pkp_global_add_f32(float *dst, const int32_t *addr, const float *vals, int64_t m,
                       void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PK_PROBE_H */
