// Non-hot kernels: initial state, population conversion, macroscopic fields
// and the FP64 global diagnostics.
//
// All of them work on the stored deviations h_i = f_i - w_i with
// w_i = prod_a W_a[c_ia] the reference equilibrium of the lattice, and use
// FP64 arithmetic. Node order is x fastest; velocity index
// i = sum_a (c_ia + 1) 3^a over the physical axes.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "elbm_codec.h"
#include "elbm_internal.h"

namespace elbm {
namespace {

__device__ __forceinline__ int cdir(int i, int a) {
  int r = i;
  for (int k = 0; k < a; ++k) r /= 3;
  return r % 3 - 1;
}

// Reference weight w_i = prod_a W_a[c_ia] in FP64.
__device__ __forceinline__ double ref_weight(const LatticeConst64& c, int i) {
  double w = 1.0;
  for (int a = 0; a < c.D; ++a) w *= c.W[a][cdir(i, a) + 1];
  return w;
}

// Triplet Psi_c(u, P, lambda) (Sec. 2.2, eqs. phi0S, phiPlusS, phiMinusS).
__device__ __forceinline__ double psi(int ci, double u, double P, double lam) {
  if (ci == 0) return 1.0 - P / (lam * lam);
  return 0.5 * (ci * u / lam + P / (lam * lam));
}

// Element index of population 0 of node `cell` (x fastest over the lattice)
// in the plane-slab layout; population i is pstride elements further on.
__device__ __forceinline__ int64_t slab_base(const LatticeConst64& c, int64_t cell) {
  const uint32_t z = uint32_t(cell) / uint32_t(c.plane);
  return int64_t(z) * c.Q * c.pstride + (cell - int64_t(z) * c.plane);
}

template <int S>
__global__ void init_kernel(LatticeConst64 c, const double* __restrict__ stage, int64_t cell0, int64_t count,
                            void* __restrict__ dstv) {
  using T = typename Raw<S>::T;
  T* dst = static_cast<T*>(dstv);
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < count;
       k += int64_t(gridDim.x) * blockDim.x) {
    const double rho = stage[k];
    double u[3], P[3];
    for (int a = 0; a < c.D; ++a) {
      u[a] = stage[(1 + a) * count + k] + c.uref[a];
      P[a] = c.T + u[a] * u[a];  // equilibrium pressure (Sec. 2.3, eq. Peqa)
    }
    const int64_t base = slab_base(c, cell0 + k);
    for (int i = 0; i < c.Q; ++i) {
      double f = rho, w = 1.0;
      for (int a = 0; a < c.D; ++a) {
        const int ci = cdir(i, a);
        f *= psi(ci, u[a], P[a], c.lam[a]);
        w *= c.W[a][ci + 1];
      }
      Raw<S>::put(dst + base + i * c.pstride, (f - w) * c.scale);
    }
  }
}

template <int S>
__global__ void pop_out_kernel(LatticeConst64 c, const void* __restrict__ srcv, int i, double* __restrict__ out) {
  using T = typename Raw<S>::T;
  const T* src = static_cast<const T*>(srcv) + i * c.pstride;
  const double w = ref_weight(c, i);
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < c.N; k += int64_t(gridDim.x) * blockDim.x)
    out[k] = w + Raw<S>::get(src + slab_base(c, k)) * c.inv_scale;
}

template <int S>
__global__ void pop_in_kernel(LatticeConst64 c, const double* __restrict__ in, int i, void* __restrict__ dstv) {
  using T = typename Raw<S>::T;
  T* dst = static_cast<T*>(dstv) + i * c.pstride;
  const double w = ref_weight(c, i);
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < c.N; k += int64_t(gridDim.x) * blockDim.x)
    Raw<S>::put(dst + slab_base(c, k), (in[k] - w) * c.scale);
}

// FP64 moments of one node of the stored state: rho and the reported
// velocity u = j/rho - g/2 (j the stored, post-force momentum).
template <int S, int D>
__device__ __forceinline__ void node_moments(const LatticeConst64& c, const typename Raw<S>::T* src, int64_t cell,
                                             double& rho, double (&u)[3]) {
  constexpr int Q = D == 3 ? 27 : 9;
  double h[Q];
  const int64_t base = slab_base(c, cell);
#pragma unroll
  for (int i = 0; i < Q; ++i) h[i] = Raw<S>::get(src + base + i * c.pstride);
  double dr = 0.0, dj[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    dr += h[i];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int ci = (i / (a == 0 ? 1 : (a == 1 ? 3 : 9))) % 3 - 1;
      if (ci > 0) dj[a] += h[i];
      if (ci < 0) dj[a] -= h[i];
    }
  }
  dr *= c.inv_scale;
  rho = 1.0 + dr;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = 0.0;
    if (a < D) u[a] = (c.uref[a] + c.lam[a] * dj[a] * c.inv_scale) / rho - 0.5 * c.g[a];
  }
}

template <int S, int D>
__global__ void field_kernel(LatticeConst64 c, const void* __restrict__ srcv, int comp, double* __restrict__ out) {
  using T = typename Raw<S>::T;
  const T* src = static_cast<const T*>(srcv);
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < c.N; k += int64_t(gridDim.x) * blockDim.x) {
    double rho, u[3];
    node_moments<S, D>(c, src, k, rho, u);
    out[k] = comp == 0 ? rho : u[comp - 1];
  }
}

// ---- deterministic FP64 block reductions ----
constexpr int kDiagThreads = 256;

struct Acc {
  double v[kRec];
};

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, 64));
  return x;
}

// Reduces field f of every thread of the block (fixed order) into lane 0 of
// thread 0; kind 0 sum, 1 max, 2 min.
__device__ double block_reduce(double x, int kind, double* sh) {
  x = kind == 0 ? wave_sum(x) : (kind == 1 ? wave_max(x) : wave_min(x));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = x;
  __syncthreads();
  double r = sh[0];
  for (int k = 1; k < kDiagThreads / 64; ++k)
    r = kind == 0 ? r + sh[k] : (kind == 1 ? fmax(r, sh[k]) : fmin(r, sh[k]));
  return r;
}

__device__ __forceinline__ int field_kind(int f) { return f == R_MAXU ? 1 : (f == R_MINRHO ? 2 : 0); }

template <int S, int D>
__global__ void __launch_bounds__(kDiagThreads)
    diag_moments_kernel(LatticeConst64 c, const void* __restrict__ srcv, float* __restrict__ ustage,
                        double* __restrict__ partials) {
  using T = typename Raw<S>::T;
  const T* src = static_cast<const T*>(srcv);
  __shared__ double sh[kDiagThreads / 64];
  double acc[kRec];
  for (int f = 0; f < kRec; ++f) acc[f] = 0.0;
  acc[R_MAXU] = 0.0;
  acc[R_MINRHO] = 1e300;
  const int nx = c.n[0], ny = c.n[1];
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < c.N; k += int64_t(gridDim.x) * blockDim.x) {
    double rho, u[3];
    node_moments<S, D>(c, src, k, rho, u);
    const bool finite = isfinite(rho) && isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]);
    acc[R_NAN] += finite ? 0.0 : 1.0;
    acc[R_MASS] += rho;
    acc[R_MOM0] += rho * u[0];
    acc[R_MOM1] += rho * u[1];
    acc[R_MOM2] += rho * u[2];
    acc[R_KE] += u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    acc[R_MINRHO] = fmin(acc[R_MINRHO], finite ? rho : -1e300);
    for (int a = 0; a < 3; ++a) ustage[a * c.N + k] = float(u[a]);
    if (c.has_mode) {
      const int64_t x = k % nx, y = (k / nx) % ny, z = k / (int64_t(nx) * ny);
      const double ph = c.mode_k[0] * (x * c.lam[0]) + c.mode_k[1] * (y * c.lam[1]) + c.mode_k[2] * (z * c.lam[2]);
      const double up = c.mode_dir[0] * u[0] + c.mode_dir[1] * u[1] + c.mode_dir[2] * u[2];
      double sn, cs;
      sincos(ph, &sn, &cs);
      acc[R_MODE_RE] += up * cs;
      acc[R_MODE_IM] -= up * sn;
      acc[R_MAXU] = fmax(acc[R_MAXU], fabs(up));
    }
  }
  for (int f = 1; f < R_USED; ++f) {
    if (f == R_ENS) continue;
    const double r = block_reduce(acc[f], field_kind(f), sh);
    if (threadIdx.x == 0) partials[blockIdx.x * kRec + f] = r;
  }
}

// Central difference of velocity component comp along axis b at the node of
// linear index `own` and coordinate pb along b (stride st, extent n), times
// 1 / (2 lambda_b) = h; periodic wrap, or the no-slip ghost u(-1) = -u(0) on a
// wall axis. FP32: the staged velocities are FP32 already, and one rounding
// of the difference keeps ~1e-7 relative accuracy per node.
__device__ __forceinline__ float dudx(const LatticeConst64& c, const float* __restrict__ u, int comp, int b, int pb,
                                      int n, int64_t own, int64_t st, float h) {
  const float* uc = u + comp * c.N;
  const float uo = uc[own];
  float up, um;
  if (pb + 1 < n) up = uc[own + st];
  else up = c.wall[b] ? -uo : uc[own - (n - 1) * st];
  if (pb > 0) um = uc[own - st];
  else um = c.wall[b] ? -uo : uc[own + (n - 1) * st];
  return (up - um) * h;
}

// Enstrophy partial sums: a block takes whole x rows (grid-strided over the
// rows), its threads the nodes of a row, so that coordinates come from one
// 32-bit division per row and every read is a coalesced row segment. The
// vorticity of a node is formed in FP32, its square accumulated in FP64.
__global__ void __launch_bounds__(kDiagThreads)
    diag_curl_kernel(LatticeConst64 c, const float* __restrict__ ustage, double* __restrict__ partials) {
  __shared__ double sh[kDiagThreads / 64];
  double ens = 0.0;
  const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
  const int64_t sy = nx, sz = int64_t(nx) * ny;
  const float h0 = float(0.5 / c.lam[0]), h1 = float(0.5 / c.lam[1]), h2 = float(0.5 / c.lam[2]);
  const int rows = ny * nz;
  for (int r = blockIdx.x; r < rows; r += gridDim.x) {
    const int y = r % ny, z = r / ny;
    const int64_t row = sy * y + sz * z;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
      const int64_t own = row + x;
      if (c.D == 2) {
        const float wz = dudx(c, ustage, 1, 0, x, nx, own, 1, h0) - dudx(c, ustage, 0, 1, y, ny, own, sy, h1);
        ens += double(wz * wz);
      } else {
        const float wx = dudx(c, ustage, 2, 1, y, ny, own, sy, h1) - dudx(c, ustage, 1, 2, z, nz, own, sz, h2);
        const float wy = dudx(c, ustage, 0, 2, z, nz, own, sz, h2) - dudx(c, ustage, 2, 0, x, nx, own, 1, h0);
        const float wz = dudx(c, ustage, 1, 0, x, nx, own, 1, h0) - dudx(c, ustage, 0, 1, y, ny, own, sy, h1);
        ens += double(wx * wx + wy * wy + wz * wz);
      }
    }
  }
  const double r = block_reduce(ens, 0, sh);
  if (threadIdx.x == 0) partials[blockIdx.x * kRec + R_ENS] = r;
}

// One block: fixed-order reduction of the per-block partials into a record:
// the enstrophy from the nb_e records of `pens`, every other field from the
// nb_m records of `pmom`. The record goes to history[(*count) % capacity]
// and *count is incremented when capacity > 0; it always goes to `last` (the
// record after the ring).
__global__ void __launch_bounds__(kDiagThreads)
    diag_final_kernel(const double* __restrict__ pmom, int nb_m, const double* __restrict__ pens, int nb_e,
                      double* __restrict__ history, int64_t* __restrict__ count, int32_t capacity,
                      double* __restrict__ last, int64_t step, double ncells) {
  __shared__ double sh[kDiagThreads / 64];
  double rec[kRec];
  for (int f = 0; f < kRec; ++f) {
    const int kind = field_kind(f);
    const double* part = f == R_ENS ? pens : pmom;
    const int nblocks = f == R_ENS ? nb_e : nb_m;
    double x = kind == 0 ? 0.0 : (kind == 1 ? 0.0 : 1e300);
    for (int b = threadIdx.x; b < nblocks; b += kDiagThreads) {
      const double v = part[b * kRec + f];
      x = kind == 0 ? x + v : (kind == 1 ? fmax(x, v) : fmin(x, v));
    }
    rec[f] = block_reduce(x, kind, sh);
  }
  if (threadIdx.x == 0) {
    rec[R_STEP] = double(step);
    rec[R_KE] = 0.5 * rec[R_KE] / ncells;
    rec[R_ENS] = rec[R_ENS] / ncells;
    rec[R_MODE_RE] /= ncells;
    rec[R_MODE_IM] /= ncells;
    for (int f = R_USED; f < kRec; ++f) rec[f] = 0.0;
    for (int f = 0; f < kRec; ++f) last[f] = rec[f];
    if (capacity > 0) {
      const int64_t n = *count;
      double* dst = history + (n % capacity) * kRec;
      for (int f = 0; f < kRec; ++f) dst[f] = rec[f];
      *count = n + 1;
    }
  }
}

int grid_for(int64_t n, int threads) {
  const int64_t g = (n + threads - 1) / threads;
  return int(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

hipError_t launch_init(const LatticeConst64& c, const double* stage, int64_t cell0, int64_t count, void* dst,
                       hipStream_t st) {
  const int g = grid_for(count, 256);
  switch (c.storage) {
    case 0: hipLaunchKernelGGL(init_kernel<0>, dim3(g), dim3(256), 0, st, c, stage, cell0, count, dst); break;
    case 1: hipLaunchKernelGGL(init_kernel<1>, dim3(g), dim3(256), 0, st, c, stage, cell0, count, dst); break;
    case 2: hipLaunchKernelGGL(init_kernel<2>, dim3(g), dim3(256), 0, st, c, stage, cell0, count, dst); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pop_out(const LatticeConst64& c, const void* src, int i, double* out, hipStream_t st) {
  const int g = grid_for(c.N, 256);
  switch (c.storage) {
    case 0: hipLaunchKernelGGL(pop_out_kernel<0>, dim3(g), dim3(256), 0, st, c, src, i, out); break;
    case 1: hipLaunchKernelGGL(pop_out_kernel<1>, dim3(g), dim3(256), 0, st, c, src, i, out); break;
    case 2: hipLaunchKernelGGL(pop_out_kernel<2>, dim3(g), dim3(256), 0, st, c, src, i, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pop_in(const LatticeConst64& c, const double* in, int i, void* dst, hipStream_t st) {
  const int g = grid_for(c.N, 256);
  switch (c.storage) {
    case 0: hipLaunchKernelGGL(pop_in_kernel<0>, dim3(g), dim3(256), 0, st, c, in, i, dst); break;
    case 1: hipLaunchKernelGGL(pop_in_kernel<1>, dim3(g), dim3(256), 0, st, c, in, i, dst); break;
    case 2: hipLaunchKernelGGL(pop_in_kernel<2>, dim3(g), dim3(256), 0, st, c, in, i, dst); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int S>
void field_s(const LatticeConst64& c, const void* src, int comp, double* out, hipStream_t st) {
  const int g = grid_for(c.N, 256);
  if (c.D == 3)
    hipLaunchKernelGGL((field_kernel<S, 3>), dim3(g), dim3(256), 0, st, c, src, comp, out);
  else
    hipLaunchKernelGGL((field_kernel<S, 2>), dim3(g), dim3(256), 0, st, c, src, comp, out);
}

hipError_t launch_field(const LatticeConst64& c, const void* src, int comp, double* out, hipStream_t st) {
  switch (c.storage) {
    case 0: field_s<0>(c, src, comp, out, st); break;
    case 1: field_s<1>(c, src, comp, out, st); break;
    case 2: field_s<2>(c, src, comp, out, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int S>
void diag_s(const LatticeConst64& c, const void* src, float* ustage, double* partials, hipStream_t st) {
  if (c.D == 3)
    hipLaunchKernelGGL((diag_moments_kernel<S, 3>), dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, c, src, ustage,
                       partials);
  else
    hipLaunchKernelGGL((diag_moments_kernel<S, 2>), dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, c, src, ustage,
                       partials);
}

hipError_t launch_diag(const LatticeConst64& c, const void* src, float* ustage, double* partials, double* history,
                       int64_t* hist_count, int32_t capacity, double* last, int64_t step, hipStream_t st) {
  const int nb = kDiagBlocks;
  switch (c.storage) {
    case 0: diag_s<0>(c, src, ustage, partials, st); break;
    case 1: diag_s<1>(c, src, ustage, partials, st); break;
    case 2: diag_s<2>(c, src, ustage, partials, st); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_diag_tail(c, ustage, partials, nb, history, hist_count, capacity, last, step, st);
}

hipError_t launch_diag_tail(const LatticeConst64& c, const float* ustage, double* partials, int nb_moments,
                            double* history, int64_t* hist_count, int32_t capacity, double* last, int64_t step,
                            hipStream_t st) {
  if (nb_moments < 1 || nb_moments > kDiagBlocks) return hipErrorInvalidValue;
  double* pens = partials + size_t(kDiagBlocks) * kRec;
  hipLaunchKernelGGL(diag_curl_kernel, dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, c, ustage, pens);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(kDiagThreads), 0, st, partials, nb_moments, pens,
                     kDiagBlocks, history, hist_count, capacity, last, step, double(c.N));
  return hipGetLastError();
}

}  // namespace elbm
