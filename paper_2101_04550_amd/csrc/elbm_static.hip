// Fixed device scratch of the allocation-free batched runner
// (elbm_batch_run_static): the per-class descriptor tables live in one
// file-scope device array instead of memory the library allocates.
//
// The array's name is only a host-side stand-in in host code; its device
// address is looked up once per device with hipGetSymbolAddress (the first
// call of the entry point on that device, with the device current) and kept.
// The tables are written by a small kernel whose arguments carry the bytes,
// so a call needs no host staging memory either.
#include <cstring>
#include <mutex>

#include "elbm_internal.h"

namespace elbm {
namespace {

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_mu;

// Bytes per table-writing launch (kept well inside the kernel-argument limit).
constexpr uint32_t kBlobBytes = 3072;
struct Blob {
  uint32_t offset;
  uint32_t bytes;
  unsigned char data[kBlobBytes];
};

__global__ void __launch_bounds__(256) write_bytes_kernel(unsigned char* __restrict__ dst, Blob b) {
  for (uint32_t k = threadIdx.x; k < b.bytes; k += blockDim.x) dst[b.offset + k] = b.data[k];
}

}  // namespace

hipError_t static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

hipError_t launch_write_bytes(void* dst, const unsigned char* src, size_t bytes, hipStream_t st) {
  if (bytes > kStaticScratchBytes) return hipErrorInvalidValue;
  for (size_t o = 0; o < bytes; o += kBlobBytes) {
    Blob b;
    b.offset = uint32_t(o);
    b.bytes = uint32_t(bytes - o < kBlobBytes ? bytes - o : kBlobBytes);
    std::memcpy(b.data, src + o, b.bytes);
    hipLaunchKernelGGL(write_bytes_kernel, dim3(1), dim3(256), 0, st, static_cast<unsigned char*>(dst), b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace elbm
