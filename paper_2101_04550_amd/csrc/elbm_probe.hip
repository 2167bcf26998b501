// Bandwidth probe: the population traffic of one D3Q27 step without its
// arithmetic, to measure what HBM bandwidth the step's access pattern can
// reach on this device (the achievable ceiling its roofline is judged
// against, beside the 8 TB/s peak).
//
// Layout as the step kernels': plane slabs along z, Q direction arrays of
// pstride elements per slab. Each thread owns one in-plane node and marches
// along z over `chunk` planes; per plane it loads the node's Q values (from
// the neighbour x - c_i when shift != 0, with periodic wrap: the pull of the
// step) into registers, then stores them to the other buffer with
// nontemporal stores, as the step does. Occupancy is set by a dynamic LDS
// reservation: lds_bytes per block limits the resident blocks per CU.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "elbm_probe.h"

namespace {

using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc rsrc(const char* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), 0, -1, 0x00020000);
}

template <int ES>
struct Elem;
template <>
struct Elem<4> {
  __device__ static uint32_t ld(Rsrc r, uint32_t off, uint32_t so) { return __builtin_amdgcn_raw_buffer_load_b32(r, off, so, 0); }
  __device__ static void st(uint32_t v, Rsrc r, uint32_t off, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, off, so, 2);
  }
};
template <>
struct Elem<2> {
  __device__ static uint32_t ld(Rsrc r, uint32_t off, uint32_t so) { return __builtin_amdgcn_raw_buffer_load_b16(r, off, so, 0); }
  __device__ static void st(uint32_t v, Rsrc r, uint32_t off, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b16(static_cast<unsigned short>(v), r, off, so, 2);
  }
};

constexpr int Q = 27;

template <int ES, bool SHIFT>
__global__ void __launch_bounds__(512) stream_kernel(const char* __restrict__ src, char* __restrict__ dst, int nx,
                                                     int ny, int nz, int chunk, uint64_t slab_bytes, uint32_t sb) {
  const int plane = nx * ny;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int z0 = blockIdx.y * chunk;
  const int z1 = min(z0 + chunk, nz);
  if (p >= plane) return;
  const int x = p % nx, y = p / nx;
  uint32_t off[3][3];
#pragma unroll
  for (int cx = 0; cx < 3; ++cx)
#pragma unroll
    for (int cy = 0; cy < 3; ++cy) {
      int xs = x - (SHIFT ? cx - 1 : 0), ys = y - (SHIFT ? cy - 1 : 0);
      xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
      ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
      off[cx][cy] = uint32_t(xs + nx * ys) * ES;
    }
  const uint32_t own = uint32_t(p) * ES;
  for (int z = z0; z < z1; ++z) {
    Rsrc rs[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int zs = z - (SHIFT ? c - 1 : 0);
      zs = zs < 0 ? zs + nz : (zs >= nz ? zs - nz : zs);
      rs[c] = rsrc(src + uint64_t(zs) * slab_bytes);
    }
    uint32_t v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = Elem<ES>::ld(rs[i / 9], off[i % 3][(i / 3) % 3], i * sb);
    const Rsrc rd = rsrc(dst + uint64_t(z) * slab_bytes);
#pragma unroll
    for (int i = 0; i < Q; ++i) Elem<ES>::st(v[i], rd, own, i * sb);
    // as the step kernels do: the plane's stores complete before the next
    // plane's loads are issued (vmcnt(0))
    __builtin_amdgcn_s_waitcnt(0xF70);
  }
}

// Plain contiguous copy in 16-byte pieces, grid-stride, nontemporal stores:
// the best case of a read + write stream. Each thread issues U loads before
// its U stores (U pieces in flight per thread).
template <int U>
__global__ void __launch_bounds__(256) copy16_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                     uint64_t n16) {
  const Rsrc rs = rsrc(reinterpret_cast<const char*>(src));
  const Rsrc rd = rsrc(reinterpret_cast<const char*>(dst));
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t k0 = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k0 < n16; k0 += U * stride) {
    decltype(__builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0)) v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // offsets stay below 2^32 bytes for buffers under 4 GiB (checked by the
      // host); pieces past the end are not loaded
      const uint64_t k = k0 + u * stride;
      if (k < n16) v[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, uint32_t(k * 16), 0, 0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t k = k0 + u * stride;
      if (k < n16) __builtin_amdgcn_raw_buffer_store_b128(v[u], rd, uint32_t(k * 16), 0, 2);
    }
  }
}

template <int ES, bool SHIFT>
hipError_t launch(const char* src, char* dst, int nx, int ny, int nz, int chunk, size_t lds, hipStream_t st) {
  const int plane = nx * ny;
  const int64_t pstride = (int64_t(plane) + 63) / 64 * 64;
  const dim3 grid((plane + 511) / 512, (nz + chunk - 1) / chunk);
  hipLaunchKernelGGL((stream_kernel<ES, SHIFT>), grid, dim3(512), lds, st, src, dst, nx, ny, nz, chunk,
                     uint64_t(pstride) * Q * ES, uint32_t(pstride) * ES);
  return hipGetLastError();
}

}  // namespace

extern "C" int32_t elbm_probe_copy(const void* src, void* dst, size_t bytes, int32_t blocks, int32_t unroll,
                                   int32_t reps, void* hip_stream, float* ms_per_launch) {
  if (!src || !dst || !ms_per_launch || reps < 1 || blocks < 1 || bytes % 16 || bytes == 0 ||
      bytes > (size_t(1) << 32) - 16 || (unroll != 1 && unroll != 2 && unroll != 4))
    return 1;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  auto one = [&]() -> hipError_t {
    const auto* s16 = static_cast<const uint4*>(src);
    auto* d16 = static_cast<uint4*>(dst);
    const uint64_t n16 = bytes / 16;
    if (unroll == 1) hipLaunchKernelGGL(copy16_kernel<1>, dim3(blocks), dim3(256), 0, st, s16, d16, n16);
    else if (unroll == 2) hipLaunchKernelGGL(copy16_kernel<2>, dim3(blocks), dim3(256), 0, st, s16, d16, n16);
    else hipLaunchKernelGGL(copy16_kernel<4>, dim3(blocks), dim3(256), 0, st, s16, d16, n16);
    return hipGetLastError();
  };
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 2;
  hipError_t e = one();
  if (e == hipSuccess) e = hipEventRecord(a, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = one();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return 2;
  *ms_per_launch = ms / float(reps);
  return 0;
}

extern "C" int32_t elbm_probe_bytes(int32_t elem_bytes, int32_t nx, int32_t ny, int32_t nz, size_t* bytes) {
  if (!bytes || (elem_bytes != 2 && elem_bytes != 4) || nx < 3 || ny < 3 || nz < 3) return 1;
  const int64_t pstride = (int64_t(nx) * ny + 63) / 64 * 64;
  if (pstride * Q * elem_bytes >= (int64_t(1) << 32)) return 1;
  *bytes = size_t(nz) * Q * size_t(pstride) * elem_bytes;
  return 0;
}

extern "C" int32_t elbm_probe_stream(const void* src, void* dst, int32_t elem_bytes, int32_t nx, int32_t ny,
                                     int32_t nz, int32_t chunk, int32_t shift, int32_t lds_bytes, int32_t reps,
                                     void* hip_stream, float* ms_per_launch) {
  size_t need = 0;
  if (elbm_probe_bytes(elem_bytes, nx, ny, nz, &need) || !src || !dst || !ms_per_launch || reps < 1 || chunk < 1 ||
      lds_bytes < 0 || lds_bytes > 160 * 1024)
    return 1;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  auto one = [&]() -> hipError_t {
    const char* s = static_cast<const char*>(src);
    char* d = static_cast<char*>(dst);
    if (elem_bytes == 4)
      return shift ? launch<4, true>(s, d, nx, ny, nz, chunk, lds_bytes, st)
                   : launch<4, false>(s, d, nx, ny, nz, chunk, lds_bytes, st);
    return shift ? launch<2, true>(s, d, nx, ny, nz, chunk, lds_bytes, st)
                 : launch<2, false>(s, d, nx, ny, nz, chunk, lds_bytes, st);
  };
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 2;
  hipError_t e = one();  // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = one();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return 2;
  *ms_per_launch = ms / float(reps);
  return 0;
}
