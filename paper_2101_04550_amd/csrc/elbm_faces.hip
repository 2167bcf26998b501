// Open boundaries of a D2Q9 lattice (FP32, FP16 or BF16 deviation storage): Grad's-
// approximation walls, symmetry planes, velocity inlets and outlets.
//
// The lattice the step kernel advances is periodic and carries one ring of
// ghost nodes on every non-periodic face. Before each step the kernels here
// rewrite every population stored at a ghost node, so that the following
// (unchanged, periodic) pull delivers
//  * to each fluid boundary node, in place of the populations that would
//    come from outside the fluid, the values of its face's rule (kernel A:
//    boundary nodes on one face; then corner nodes, which may copy values
//    the first pass wrote);
//  * to each ghost node, populations whose density and normal momentum are
//    those of its inward neighbour (the normal momentum reversed at walls
//    and symmetry planes): the step kernel's central difference of the
//    anomaly across the face then sees an odd ghost at walls and symmetry
//    planes and an even one at inlets and outlets (kernel B).
// The rules (the paper names Grad's approximation for its walls, Sec. 3, and
// sets up the flat plate of Sec. 3.4 with an inlet, an outlet and a symmetry
// plane, without defining them): for a missing population i of boundary
// node x on a face with inward normal s e_n,
//  SYMMETRY  f_i = f'_{i*}(x - c_i,t e_t): specular reflection at the
//            halfway plane (i* has the normal component reversed);
//  WALL      f_i = Grad's approximation at the target velocity
//            u_t = (2 u_w + u_f)/3 (on the line through the wall velocity
//            at distance lambda_n/2 and the inward neighbour's velocity
//            u_f at 3 lambda_n/2), the density of the mass and
//            normal-momentum balance rho_t (1 - s u_t,n/lambda_n) =
//            S_0 + 2 S_out, and the stress rho_t (T + u_t u_t)
//            - (rho_t T/omega)(grad u_t + grad u_t^T) (under the
//            multi-relaxation-time collision the trace part of
//            grad u_t + grad u_t^T over omega_bulk instead);
//  INLET     f_i = f'_{-i}(x) + f^eq_i(rho_x, u_in) - f^eq_{-i}(rho_x, u_in):
//            bounce-back from a surface moving at u_in at the halfway plane,
//            with the equilibrium of Sec. 2.3 (eq. 27eq) at the node's own
//            density (an equilibrium set at the node itself lets
//            disturbances grow on the lambda_x = 2 lattice near omega = 2);
//  OUTLET    f_i = f^eq_i(rho_out, u_f) + f_i(x_f) - f^eq_i(rho_f, u_f): the
//            prescribed density with the inward neighbour's velocity and
//            non-equilibrium part.
// All of it in FP64 from the stored deviations (read exactly); a population
// is written back as a deviation from the reference weight, rounded once to
// the storage format.
#include "elbm.h"
#include "elbm_codec.h"
#include "elbm_internal.h"

namespace elbm {
namespace {

__device__ __forceinline__ int cdir(int i, int a) { return a == 0 ? i % 3 - 1 : i / 3 - 1; }
__device__ __forceinline__ int dir_index(int cx, int cy) { return (cx + 1) + 3 * (cy + 1); }

// Triplet Psi_c(u, P, lambda) (Sec. 2.2, eqs. phi0S, phiPlusS, phiMinusS).
__device__ __forceinline__ double tri(int c, double u, double P, double lam) {
  if (c == 0) return 1.0 - P / (lam * lam);
  return 0.5 * (c * u / lam + P / (lam * lam));
}

template <int S>
struct View {
  using T = typename Raw<S>::T;
  const FaceArgs& a;
  T* const h;
  __device__ explicit View(const FaceArgs& args) : a(args), h(static_cast<T*>(args.h)) {}
  __device__ int wrap(int v, int ax) const {
    const int n = a.N[ax];
    v %= n;
    return v < 0 ? v + n : v;
  }
  __device__ int64_t idx(int X, int Y, int i) const { return (int64_t(Y) * 9 + i) * a.pstride + X; }
  // population i stored at storage node (X, Y) (wrapped)
  __device__ double slot(int X, int Y, int i) const {
    return a.w[i] + Raw<S>::get(h + idx(wrap(X, 0), wrap(Y, 1), i)) * a.inv_scale;
  }
  __device__ void set_slot(int X, int Y, int i, double f) const {
    Raw<S>::put(h + idx(wrap(X, 0), wrap(Y, 1), i), (f - a.w[i]) * a.scale);
  }
  // fluid coordinates -> storage coordinates
  __device__ int SX(int x) const { return x + a.o[0]; }
  __device__ int SY(int y) const { return y + a.o[1]; }
  // whether fluid node (x, y) exists (a periodic axis wraps)
  __device__ bool fluid(int x, int y) const {
    return (a.o[0] == 0 || (x >= 0 && x < a.n[0])) && (a.o[1] == 0 || (y >= 0 && y < a.n[1]));
  }
  // post-collision density and reported velocity j'/rho - g/2 of fluid node (x, y)
  __device__ void state(int x, int y, double& rho, double (&u)[2]) const {
    double r = 0.0, j[2] = {0.0, 0.0};
    for (int i = 0; i < 9; ++i) {
      const double f = slot(SX(x), SY(y), i);
      r += f;
      j[0] += cdir(i, 0) * f;
      j[1] += cdir(i, 1) * f;
    }
    rho = r;
    for (int b = 0; b < 2; ++b) u[b] = a.lam[b] * j[b] / r - 0.5 * a.g[b];
  }
};

// Rule of a boundary node: fills fm[i] for its missing directions.
template <int S>
__device__ void boundary_rule(const View<S>& v, const FaceNode& nd, double (&fm)[9], bool (&miss)[9]) {
  const FaceArgs& A = v.a;
  const int x = nd.x, y = nd.y, F = nd.face, kind = nd.kind;
  const int n_ax = F >> 1, t_ax = 1 - n_ax;
  const int s = (F & 1) ? -1 : 1;
  const int xf = n_ax == 0 ? x + s : x, yf = n_ax == 1 ? y + s : y;
  for (int i = 0; i < 9; ++i) miss[i] = !v.fluid(x - cdir(i, 0), y - cdir(i, 1));

  if (kind == ELBM_FACE_SYMMETRY) {
    for (int i = 0; i < 9; ++i) {
      if (!miss[i]) continue;
      const int ct = cdir(i, t_ax);
      const int sx = t_ax == 0 ? x - ct : x, sy = t_ax == 1 ? y - ct : y;
      const int mi = n_ax == 0 ? dir_index(-cdir(i, 0), cdir(i, 1)) : dir_index(cdir(i, 0), -cdir(i, 1));
      fm[i] = v.slot(v.SX(sx), v.SY(sy), mi);
    }
  } else if (kind == ELBM_FACE_WALL) {
    double rf, uf[2];
    v.state(xf, yf, rf, uf);
    double uw[2] = {0.0, 0.0};
    uw[t_ax] = A.wall_u[F];
    double ut[2];
    for (int b = 0; b < 2; ++b) ut[b] = (2.0 * uw[b] + uf[b]) / 3.0;
    double S0 = 0.0, Sout = 0.0;
    for (int i = 0; i < 9; ++i) {
      if (miss[i]) continue;
      const double f = v.slot(v.SX(x) - cdir(i, 0), v.SY(y) - cdir(i, 1), i);
      if (cdir(i, n_ax) == 0) S0 += f;
      if (cdir(i, n_ax) == -s) Sout += f;
    }
    const double rt = (S0 + 2.0 * Sout) / (1.0 - s * ut[n_ax] / A.lam[n_ax]);
    // grad[a][b] = d u_b / d x_a
    double grad[2][2];
    for (int b = 0; b < 2; ++b) grad[n_ax][b] = s * (uf[b] - uw[b]) / (1.5 * A.lam[n_ax]);
    double rp, up[2], rm, um[2];
    v.state(t_ax == 0 ? xf + 1 : xf, t_ax == 1 ? yf + 1 : yf, rp, up);
    v.state(t_ax == 0 ? xf - 1 : xf, t_ax == 1 ? yf - 1 : yf, rm, um);
    for (int b = 0; b < 2; ++b) grad[t_ax][b] = (up[b] - um[b]) / (2.0 * A.lam[t_ax]) / 3.0;
    // Pi_neq = -rho_t T (S_dev / omega + S_iso / omega_bulk), S = grad u + grad u^T,
    // S_iso = m I with m = (S_xx + S_yy) / 2 (omega_bulk = omega under LBGK)
    const double m = grad[0][0] + grad[1][1];
    const double kd = -(rt * A.T / A.omega), kb = -(rt * A.T / A.omega_bulk);
    const double pxx = kd * (2.0 * grad[0][0] - m) + kb * m, pyy = kd * (2.0 * grad[1][1] - m) + kb * m;
    const double pxy = kd * (grad[0][1] + grad[1][0]);
    const double Px = A.T + ut[0] * ut[0] + pxx / rt, Py = A.T + ut[1] * ut[1] + pyy / rt;
    for (int i = 0; i < 9; ++i) {
      if (!miss[i]) continue;
      const int cx = cdir(i, 0), cy = cdir(i, 1);
      fm[i] = rt * tri(cx, ut[0], Px, A.lam[0]) * tri(cy, ut[1], Py, A.lam[1]) +
              cx * cy * pxy / (4.0 * A.lam[0] * A.lam[1]);
    }
  } else if (kind == ELBM_FACE_INLET) {
    double rx, ux0[2];
    v.state(x, y, rx, ux0);
    const double ux = A.inlet_u[F][0], uy = A.inlet_u[F][1];
    const double Px = A.T + ux * ux, Py = A.T + uy * uy;  // equilibrium pressure (Sec. 2.3, eq. Peqa)
    for (int i = 0; i < 9; ++i) {
      if (!miss[i]) continue;
      const int cx = cdir(i, 0), cy = cdir(i, 1);
      const double fe = rx * tri(cx, ux, Px, A.lam[0]) * tri(cy, uy, Py, A.lam[1]);
      const double fo = rx * tri(-cx, ux, Px, A.lam[0]) * tri(-cy, uy, Py, A.lam[1]);
      fm[i] = v.slot(v.SX(x), v.SY(y), 8 - i) + fe - fo;
    }
  } else {  // ELBM_FACE_OUTLET (the neighbour's pulled values are complete after the first pass)
    double rf, uf[2];
    v.state(xf, yf, rf, uf);
    const double Px = A.T + uf[0] * uf[0], Py = A.T + uf[1] * uf[1];
    const double ro = A.outlet_rho[F];
    for (int i = 0; i < 9; ++i) {
      if (!miss[i]) continue;
      const int cx = cdir(i, 0), cy = cdir(i, 1);
      const double e = tri(cx, uf[0], Px, A.lam[0]) * tri(cy, uf[1], Py, A.lam[1]);
      fm[i] = ro * e + v.slot(v.SX(xf) - cx, v.SY(yf) - cy, i) - rf * e;
    }
  }
}

// Kernel A: one thread per boundary node of [first, first + count).
template <int S>
__global__ void faces_boundary_kernel(FaceArgs A, int first, int count) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const View<S> v(A);
  const FaceNode nd = A.nodes[first + k];
  double fm[9];
  bool miss[9];
  boundary_rule(v, nd, fm, miss);
  // write the missing values into the ghost slots they are pulled from, and
  // keep the node's pulled moments for the ghosts' anomaly
  const int X = v.SX(nd.x), Y = v.SY(nd.y);
  double r = 0.0, j[2] = {0.0, 0.0};
  for (int i = 0; i < 9; ++i) {
    const int cx = cdir(i, 0), cy = cdir(i, 1);
    double f;
    if (miss[i]) {
      f = fm[i];
      v.set_slot(X - cx, Y - cy, i, f);
    } else {
      f = v.slot(X - cx, Y - cy, i);
    }
    r += f;
    j[0] += cx * f;
    j[1] += cy * f;
  }
  double* m = A.mom + 3 * (first + k);
  m[0] = r;
  m[1] = A.lam[0] * j[0];
  m[2] = A.lam[1] * j[1];
}

// Kernel B: one thread per ghost node: its populations that come from other
// ghost nodes are set to w_i (a + b c_in) so that, with those that come from
// fluid nodes, its pulled density and normal momentum hit the targets.
template <int S>
__global__ void faces_ghost_kernel(FaceArgs A) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= A.n_ghost) return;
  const View<S> v(A);
  const FaceGhost gh = A.ghosts[k];
  const int ax = gh.axis;
  double rt = 1.0, jt = 0.0;
  if (gh.node >= 0) {
    rt = A.mom[3 * gh.node];
    jt = gh.parity * A.mom[3 * gh.node + 1 + ax];
  }
  double su = 0.0, sju = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
  bool ctl[9];
  for (int i = 0; i < 9; ++i) {
    const int cx = cdir(i, 0), cy = cdir(i, 1);
    const int SXs = v.wrap(gh.X - cx, 0), SYs = v.wrap(gh.Y - cy, 1);
    const bool from_fluid =
        (A.o[0] == 0 || (SXs >= 1 && SXs <= A.n[0])) && (A.o[1] == 0 || (SYs >= 1 && SYs <= A.n[1]));
    ctl[i] = !from_fluid;
    const int cn = cdir(i, ax);
    if (from_fluid) {
      const double f = v.slot(SXs, SYs, i);
      su += f;
      sju += cn * f;
    } else {
      s0 += A.w[i];
      s1 += A.w[i] * cn;
      s2 += A.w[i] * cn * cn;
    }
  }
  const double R = rt - su, J = jt / A.lam[ax] - sju;
  const double det = s0 * s2 - s1 * s1;
  const double ca = (R * s2 - J * s1) / det, cb = (s0 * J - s1 * R) / det;
  for (int i = 0; i < 9; ++i)
    if (ctl[i]) v.set_slot(gh.X - cdir(i, 0), gh.Y - cdir(i, 1), i, A.w[i] * (ca + cb * cdir(i, ax)));
}

template <int S>
hipError_t launch_s(const FaceArgs& A, hipStream_t st) {
  constexpr int NT = 128;
  if (A.n_single > 0) {
    hipLaunchKernelGGL(faces_boundary_kernel<S>, dim3((A.n_single + NT - 1) / NT), dim3(NT), 0, st, A, 0,
                       A.n_single);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (A.n_corner > 0) {
    hipLaunchKernelGGL(faces_boundary_kernel<S>, dim3((A.n_corner + NT - 1) / NT), dim3(NT), 0, st, A, A.n_single,
                       A.n_corner);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (A.n_ghost > 0) {
    hipLaunchKernelGGL(faces_ghost_kernel<S>, dim3((A.n_ghost + NT - 1) / NT), dim3(NT), 0, st, A);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_faces(const FaceArgs& A, hipStream_t st) {
  switch (A.storage) {
    case 0: return launch_s<0>(A, st);
    case 1: return launch_s<1>(A, st);
    case 2: return launch_s<2>(A, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace elbm
