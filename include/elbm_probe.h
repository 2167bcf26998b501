/*
 * elbm_probe.h -- bandwidth probe of the extended-LBGK step's memory traffic
 * (libelbm_probe.so; measurement only, not part of the method).
 *
 * elbm_probe_stream moves the populations of a D3Q27 lattice exactly as one
 * step does -- 27 loads per node from the plane-slab layout (optionally from
 * the pulled neighbours x - c_i, periodic) and 27 nontemporal stores to the
 * other buffer, the plane's memory operations completed before the next
 * plane's are issued -- without any arithmetic, so its bandwidth is the
 * ceiling of the step's access pattern on this device; elbm_probe_copy is a
 * plain 16-byte-wide copy, the best case of a read + write stream.
 */
#ifndef ELBM_PROBE_H
#define ELBM_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of one population buffer of an nx x ny x nz D3Q27 lattice with
 * elem_bytes (2 or 4) per value, plane slabs padded to 64 elements per
 * direction array. Returns 0, or 1 on invalid arguments. Host only. */
int32_t elbm_probe_bytes(int32_t elem_bytes, int32_t nx, int32_t ny, int32_t nz, size_t* bytes);

/* Runs `reps` timed launches (after one untimed) that copy device buffer
 * `src` to `dst` (both elbm_probe_bytes long, caller-owned) population by
 * population: each thread owns one in-plane node and marches over `chunk`
 * planes; shift != 0 pulls from x - c_i as the step does. lds_bytes (0 to
 * 160 KiB) of dynamic LDS per 512-thread block limit the resident blocks per
 * CU (the step kernels' occupancy can be mimicked). *ms_per_launch receives
 * the mean launch time (HIP events on `hip_stream`). Returns 0, 1 on invalid
 * arguments, 2 on a HIP error. Synchronises the stream. */
int32_t elbm_probe_stream(const void* src, void* dst, int32_t elem_bytes, int32_t nx, int32_t ny, int32_t nz,
                          int32_t chunk, int32_t shift, int32_t lds_bytes, int32_t reps, void* hip_stream,
                          float* ms_per_launch);

/* Plain device copy of `bytes` (a multiple of 16, below 4 GiB) from `src` to
 * `dst` in 16-byte pieces with nontemporal stores, `blocks` blocks of 256
 * threads striding over the buffer, each thread issuing `unroll` (1, 2 or 4)
 * loads before its stores: the best case of a read + write stream. Times
 * `reps` launches after one untimed as elbm_probe_stream does. */
int32_t elbm_probe_copy(const void* src, void* dst, size_t bytes, int32_t blocks, int32_t unroll, int32_t reps,
                        void* hip_stream, float* ms_per_launch);

#ifdef __cplusplus
}
#endif

#endif /* ELBM_PROBE_H */
