// Grad's-approximation walls on the y faces of a D3Q27 lattice, x and z
// periodic: the walls Sec. 3 names for the wall-bounded cases, in the
// channel geometry of Sec. 3.5. The three-dimensional form of the D2Q9 wall
// of elbm_faces.hip. The fluid rows are storage rows 1 .. n_y; rows 0 and
// n_y + 1 are ghost rows that the step kernel pulls from, rewritten before
// every step by three kernels:
//  U (one thread per wall node) records the reported velocity u_f of the
//    node's inward neighbour;
//  A (one thread per wall node) sets the populations a boundary node pulls
//    from beyond its wall (c_y = s, s = +1 at the low wall, -1 at the high
//    one) to Grad's approximation at the target velocity u_t = (2 u_w + u_f)/3
//    (u_f: the inward neighbour's velocity), the density rho_t of the mass
//    and normal-momentum balance rho_t (1 - s u_t,y/lambda_y) = S_0 + 2 S_out
//    and the stress rho_t (T + u_t u_t) + Pi_neq, Pi_neq = -rho_t T
//    (S_dev/omega + S_iso/omega_bulk), S = grad u_t + grad u_t^T (along y
//    s (u_f - u_w)/(3 lambda_y/2), along x and z central differences of u_f
//    over 3; omega_bulk = omega under LBGK):
//      f_i = rho_t prod_a Psi_a + sum_{a<b} c_a c_b Pi_neq,ab/(4 lambda_a lambda_b) Psi_d;
//  B (one thread per ghost node) sets the ghost's other inbound populations
//    to w_i (a + b c_iy) so that its pulled density and normal momentum are
//    rho and -j_y of the boundary node it faces: the anomaly difference at
//    the boundary row then sees an odd ghost, as next to a bounce-back wall.
// Each ghost slot is written by one thread (A: the directions with c_y = s
// of the row beyond the wall; B: the others), and no kernel reads a ghost
// row. FP64 arithmetic on the stored deviations (FP32, or FP16 / BF16
// storage, read exactly and rounded once when written).
#include "elbm_codec.h"
#include "elbm_internal.h"

namespace elbm {
namespace {

__device__ __forceinline__ int c3(int i, int a) { return a == 0 ? i % 3 - 1 : (a == 1 ? (i / 3) % 3 - 1 : i / 9 - 1); }

// Triplet Psi_c(u, P, lambda) (Sec. 2.2, eqs. phi0S, phiPlusS, phiMinusS).
__device__ __forceinline__ double tri(int c, double u, double P, double lam) {
  if (c == 0) return 1.0 - P / (lam * lam);
  return 0.5 * (c * u / lam + P / (lam * lam));
}

template <int S>
struct View3 {
  using T = typename Raw<S>::T;
  const Walls3Args& a;
  T* const h;
  __device__ explicit View3(const Walls3Args& args) : a(args), h(static_cast<T*>(args.h)) {}
  // periodic index of a coordinate at most one period outside the storage
  // (every caller offsets an in-range coordinate by -1, 0 or +1)
  __device__ int wrap(int v, int ax) const {
    const int n = a.N[ax];
    return v < 0 ? v + n : (v >= n ? v - n : v);
  }
  __device__ int64_t idx(int X, int Y, int Z, int i) const {
    return (int64_t(wrap(Z, 2)) * 27 + i) * a.pstride + wrap(X, 0) + int64_t(a.N[0]) * wrap(Y, 1);
  }
  __device__ double slot(int X, int Y, int Z, int i) const {
    return a.w[i] + Raw<S>::get(h + idx(X, Y, Z, i)) * a.inv_scale;
  }
  __device__ void set_slot(int X, int Y, int Z, int i, double f) const {
    Raw<S>::put(h + idx(X, Y, Z, i), (f - a.w[i]) * a.scale);
  }
  // reported velocity (j' - rho g/2)/rho of the post-collision state at a storage node
  __device__ void velocity(int X, int Y, int Z, double (&u)[3]) const {
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const double f = slot(X, Y, Z, i);
      r += f;
      for (int b = 0; b < 3; ++b) j[b] += c3(i, b) * f;
    }
    for (int b = 0; b < 3; ++b) u[b] = a.lam[b] * j[b] / r - 0.5 * a.g[b];
  }
};

// Kernel A: one thread per wall node, the low face (k < n_x n_z) then the high one.
constexpr int kWallThreads = 128;

// Kernel U: one thread per wall node (indexed as in kernel A), the reported
// velocity of its inward neighbour, which kernel A reads for the node itself
// and for its four neighbours along the wall.
template <int S>
__global__ void __launch_bounds__(kWallThreads) walls3_inward_kernel(Walls3Args A) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(A.n[0]) * A.n[2];
  if (k >= 2 * per) return;
  const View3<S> v(A);
  const int F = int(k / per);
  const int64_t r = k - F * per;
  const int X = int(r % A.n[0]), Z = int(r / A.n[0]);
  const int Yf = F == 0 ? 2 : A.n[1] - 1;
  double u[3];
  v.velocity(X, Yf, Z, u);
  for (int b = 0; b < 3; ++b) A.uin[3 * k + b] = u[b];
}

template <int S>
__global__ void __launch_bounds__(kWallThreads) walls3_boundary_kernel(Walls3Args A) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(A.n[0]) * A.n[2];
  if (k >= 2 * per) return;
  const View3<S> v(A);
  const int F = int(k / per);
  const int64_t r = k - F * per;
  const int X = int(r % A.n[0]), Z = int(r / A.n[0]);
  const int s = F == 0 ? 1 : -1;
  const int Y = F == 0 ? 1 : A.n[1];  // storage row of the boundary node
  double uf[3], uw[3] = {F == 0 ? A.wall_u[0] : A.wall_u[1], 0.0, 0.0}, ut[3];
  // inward-row velocity of wall node (x, z) of this face, from kernel U
  auto inward = [&](int x, int z, double (&u)[3]) {
    x = x < 0 ? x + A.n[0] : (x >= A.n[0] ? x - A.n[0] : x);
    z = z < 0 ? z + A.n[2] : (z >= A.n[2] ? z - A.n[2] : z);
    const double* q = A.uin + 3 * (F * per + int64_t(z) * A.n[0] + x);
    for (int b = 0; b < 3; ++b) u[b] = q[b];
  };
  inward(X, Z, uf);
  for (int b = 0; b < 3; ++b) ut[b] = (2.0 * uw[b] + uf[b]) / 3.0;
  double S0 = 0.0, Sout = 0.0;
  #pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int cy = c3(i, 1);
    if (cy == s) continue;
    const double f = v.slot(X - c3(i, 0), Y - cy, Z - c3(i, 2), i);
    if (cy == 0) S0 += f;
    else Sout += f;
  }
  const double rt = (S0 + 2.0 * Sout) / (1.0 - s * ut[1] / A.lam[1]);
  // grad[a][b] = d u_b / d x_a
  double grad[3][3], up[3], um[3];
  for (int b = 0; b < 3; ++b) grad[1][b] = s * (uf[b] - uw[b]) / (1.5 * A.lam[1]);
  inward(X + 1, Z, up);
  inward(X - 1, Z, um);
  for (int b = 0; b < 3; ++b) grad[0][b] = (up[b] - um[b]) / (2.0 * A.lam[0]) / 3.0;
  inward(X, Z + 1, up);
  inward(X, Z - 1, um);
  for (int b = 0; b < 3; ++b) grad[2][b] = (up[b] - um[b]) / (2.0 * A.lam[2]) / 3.0;
  // Pi_neq = -rho_t T (S_dev / omega + S_iso / omega_bulk), S_iso = (tr S / 3) I
  const double m = 2.0 * (grad[0][0] + grad[1][1] + grad[2][2]) / 3.0;
  const double kd = -(rt * A.T / A.omega), kb = -(rt * A.T / A.omega_bulk);
  double Pi[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const double sab = grad[a][b] + grad[b][a];
      Pi[a][b] = a == b ? kd * (sab - m) + kb * m : kd * sab;
    }
  double P[3];
  for (int a = 0; a < 3; ++a) P[a] = A.T + ut[a] * ut[a] + Pi[a][a] / rt;
  double rho_b = 0.0, jy_b = 0.0;
  #pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int cx = c3(i, 0), cy = c3(i, 1), cz = c3(i, 2);
    double f;
    if (cy == s) {
      const double px = tri(cx, ut[0], P[0], A.lam[0]), py = tri(cy, ut[1], P[1], A.lam[1]);
      const double pz = tri(cz, ut[2], P[2], A.lam[2]);
      f = rt * px * py * pz + cx * cy * Pi[0][1] / (4.0 * A.lam[0] * A.lam[1]) * pz +
          cx * cz * Pi[0][2] / (4.0 * A.lam[0] * A.lam[2]) * py + cy * cz * Pi[1][2] / (4.0 * A.lam[1] * A.lam[2]) * px;
      v.set_slot(X - cx, Y - cy, Z - cz, i, f);
    } else {
      f = v.slot(X - cx, Y - cy, Z - cz, i);
    }
    rho_b += f;
    jy_b += cy * f;
  }
  A.mom[2 * k] = rho_b;
  A.mom[2 * k + 1] = A.lam[1] * jy_b;
}

// Kernel B: one thread per ghost node, the low ghost row (k < n_x n_z) then the high one.
template <int S>
__global__ void __launch_bounds__(kWallThreads) walls3_ghost_kernel(Walls3Args A) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(A.n[0]) * A.n[2];
  if (k >= 2 * per) return;
  const View3<S> v(A);
  const int F = int(k / per);
  const int64_t r = k - F * per;
  const int X = int(r % A.n[0]), Z = int(r / A.n[0]);
  const int G = F == 0 ? 0 : A.n[1] + 1;
  const double rt = A.mom[2 * k], jt = -A.mom[2 * k + 1];  // odd ghost of the boundary node
  double su = 0.0, sju = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
  #pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int cy = c3(i, 1);
    const int Ys = v.wrap(G - cy, 1);
    if (Ys >= 1 && Ys <= A.n[1]) {
      const double f = v.slot(X - c3(i, 0), Ys, Z - c3(i, 2), i);
      su += f;
      sju += cy * f;
    } else {
      s0 += A.w[i];
      s1 += A.w[i] * cy;
      s2 += A.w[i] * cy * cy;
    }
  }
  const double R = rt - su, J = jt / A.lam[1] - sju;
  const double det = s0 * s2 - s1 * s1;
  const double ca = (R * s2 - J * s1) / det, cb = (s0 * J - s1 * R) / det;
  #pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int cy = c3(i, 1);
    const int Ys = v.wrap(G - cy, 1);
    if (!(Ys >= 1 && Ys <= A.n[1])) v.set_slot(X - c3(i, 0), Ys, Z - c3(i, 2), i, A.w[i] * (ca + cb * cy));
  }
}

template <int S>
hipError_t launch_s(const Walls3Args& A, hipStream_t st) {
  constexpr int NT = kWallThreads;
  const int64_t count = 2 * int64_t(A.n[0]) * A.n[2];
  const int blocks = int((count + NT - 1) / NT);
  hipLaunchKernelGGL(walls3_inward_kernel<S>, dim3(blocks), dim3(NT), 0, st, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(walls3_boundary_kernel<S>, dim3(blocks), dim3(NT), 0, st, A);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(walls3_ghost_kernel<S>, dim3(blocks), dim3(NT), 0, st, A);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_walls3(const Walls3Args& A, hipStream_t st) {
  switch (A.storage) {
    case 0: return launch_s<0>(A, st);
    case 1: return launch_s<1>(A, st);
    case 2: return launch_s<2>(A, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace elbm
