// Fused extended-LBGK step kernels for gfx950.
//
// One launch advances every tile of every lattice in a descriptor table by one
// time step (Sec. 2.1, eq. LBGK). Per node the kernel
//   1. pulls the post-collision populations of the previous step,
//      f_i(x) = f'_i(x - c_i), with halfway bounce-back on wall axes;
//   2. forms rho and j = rho u (Sec. 2.1, eqs. density, momentum);
//   3. forms the diagonal anomaly Q~_a = j_a (lambda_a^2 - 3T) - j_a^3/rho^2
//      (Sec. 2.3, eq. Deviation) at the node and at its axis neighbours;
//   4. takes the second-order central difference of Q~_a along a with node
//      spacing lambda_a (Sec. 2.3, eq. Paastar1);
//   5. sets P*_a = T + u_a^2 + (2 - w)/(2 rho w) dQ~_a (Sec. 2.4, eq. Paastar);
//   6. builds f*_i = rho prod_a Psi_{c_ia}(u_a, P*_a, lambda_a) (Sec. 2.2,
//      eqs. phi0S, phiPlusS, phiMinusS, prod; Sec. 2.3, eq. 27eqext);
//   7. relaxes f'_i = f_i + w (f*_i - f_i) and adds the exact-difference body
//      force F_i = f^eq_i(rho, u + g) - f^eq_i(rho, u); stores f'.
//
// Layout and schedule
// -------------------
// Populations are stored in plane slabs along the slowest axis (plane z: Q
// direction arrays of the plane's nodes, x fastest), two buffers (ping-pong).
// A block owns a tile of the x-y plane (D3Q27) or an x strip (D2Q9) and
// marches along the slowest axis (z, resp. y) over `chunk` planes. The
// anomaly of the marched axis comes from a three-plane register ring
// (previous, current, next); the anomalies of the tiled axes go through LDS,
// double buffered by plane, with a one-node cross halo whose nodes are
// pulled by the first threads of the block. Each plane costs one HBM read
// and one HBM write of every population of its nodes; halo and ring-end pulls
// re-read data neighbouring tiles also read (L2).
//
// Two kernels implement the march:
//   step_kernel     -- register pull: a thread loads each of its node's Q
//                      values with one buffer load (64 x 8 tiles, 512 threads;
//                      D2Q9 strips of 256); every lattice class.
//   step_kernel_lds -- LDS staged (16-bit storage, D3Q27, full 64 x 16 tiles,
//                      x and z periodic, y periodic or bounce-back; 1024
//                      threads): the block stages the rows its tile pulls
//                      from with direct buffer-to-LDS loads and pulls from
//                      LDS.
// Both run the same per-node arithmetic (collide) on the same stored values.
// Tiles of odd chunks march down the slowest axis, so that two chunks read
// the planes at their common face at about the same time.
//
// Arithmetic is FP32 on deviations h_i = f_i - w_i from the reference
// equilibrium w_i = prod_a W_a[c_ia] (rho = 1, u = u_ref). Moments,
// velocities, the pressure and the triplets are carried as deviations from
// their reference values and the product form as
//   prod_a (W_a + d_a) - prod_a W_a
//     = ((d_0 p_1 + W_0 d_1) p_2 + W_0 W_1 d_2)     (p_a = W_a + d_a),
// so that every rounding error is relative to the (small) deviation rather
// than to the population itself.
//
// Tiles are mapped to blocks XCD-contiguously: the hardware deals
// consecutive workgroups round-robin over the 8 XCDs, so block b serves the
// (b mod 8)-th contiguous eighth of the tile range. Neighbouring tiles then
// run on one XCD at about the same time and their halo re-reads hit its L2.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <type_traits>

#include "elbm_internal.h"

namespace elbm {
namespace {

// Population arrays are accessed through buffer resources: a uniform base
// address (direction and plane, in scalar registers) plus a 32-bit per-lane
// byte offset that stays fixed along the march. Bounds checking is left open
// (num_records = 2^32 - 1); every offset is in range by construction. A
// resource of zero records is the one exception: the hardware's range check
// drops every store through it (the staged kernel's rows beyond n_y).
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc rsrc(const char* base, int num_records = -1) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), 0, num_records, 0x00020000);
}
constexpr int kNonTemporal = 2;  // cache policy of the stores: no reuse before the next launch

// Storage formats through their raw bits: FP32 values, or the 16 bits of an
// FP16 / BF16 value (deviations scaled by the lattice's storage scale).
template <int S>
struct Store;

template <>
struct Store<0> {
  using T = float;
  using R = float;
  __device__ static __forceinline__ R load(Rsrc r, uint32_t off, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
  }
  __device__ static __forceinline__ float to_float(R r) { return r; }
  __device__ static __forceinline__ void store(Rsrc r, uint32_t off, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, soff, kNonTemporal);
  }
};

template <>
struct Store<1> {
  using T = __half;
  using R = unsigned short;
  __device__ static __forceinline__ R load(Rsrc r, uint32_t off, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0);
  }
  __device__ static __forceinline__ float to_float(R r) { return __half2float(__ushort_as_half(r)); }
  __device__ static __forceinline__ void store(Rsrc r, uint32_t off, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), r, off, soff, kNonTemporal);
  }
};

template <>
struct Store<2> {
  using T = __hip_bfloat16;
  using R = unsigned short;
  __device__ static __forceinline__ R load(Rsrc r, uint32_t off, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0);
  }
  __device__ static __forceinline__ float to_float(R r) { return __uint_as_float(unsigned(r) << 16); }
  __device__ static __forceinline__ void store(Rsrc r, uint32_t off, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(__bfloat16_as_ushort(__float2bfloat16(v)), r, off, soff, kNonTemporal);
  }
};

// Waits until this wave's vector-memory operations (loads and stores) are
// complete: vmcnt(0), expcnt and lgkmcnt left open (gfx9 encoding).
__device__ __forceinline__ void drain_vm() { __builtin_amdgcn_s_waitcnt(0xF70); }
// ... and its LDS / scalar-memory operations as well.
__device__ __forceinline__ void drain_all() { __builtin_amdgcn_s_waitcnt(0); }
// Waits until at most 27 vector-memory operations of this wave are in flight:
// the counter retires in issue order, so after the 27 stores of a D3Q27 node
// every earlier load is complete while the stores may still be in flight
// (vmcnt(27): low bits 0xB, high bits 0x4000; expcnt and lgkmcnt open).
__device__ __forceinline__ void wait_vm_but_stores() { __builtin_amdgcn_s_waitcnt(0x4F7B); }

// 1/x with the hardware reciprocal (1 ulp).
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Velocity component of direction i along an internal axis. Directions are
// numbered lexicographically over the lattice's own axes:
// D3Q27 i = (cx+1) + 3 (cy+1) + 9 (cz+1); D2Q9 i = (cx+1) + 3 (cy+1), whose
// y is internal axis 2.
template <int D>
__host__ __device__ constexpr int cq(int i, int ax) {
  return D == 3 ? (ax == 0 ? i % 3 - 1 : (ax == 1 ? (i / 3) % 3 - 1 : i / 9 - 1))
                : (ax == 0 ? i % 3 - 1 : (ax == 1 ? 0 : i / 3 - 1));
}

template <int D, int S>
struct Geo {
  static constexpr int Q = D == 3 ? 27 : 9;
  static constexpr int TXW = D == 3 ? kTileX3 : 64 * kStrips2;  // tile width (x)
  static constexpr int TYR = D == 3 ? kRows3 : 1;               // tile rows (axis 1)
  static constexpr int NT = TXW * TYR;                          // threads per block
  static constexpr int HY = D == 3 ? 2 * TXW : 0;               // axis-1 halo nodes
  static constexpr int HX = 2 * TYR;                            // axis-0 halo nodes
  static constexpr int LX = TYR * (TXW + 2);                    // LDS floats, axis 0
  static constexpr int LY = D == 3 ? (TYR + 2) * TXW : 0;       // LDS floats, axis 1
  static constexpr int LDS = 2 * (LX + LY);
};

template <int D>
struct Threads {
  static constexpr int value = Geo<D, 0>::NT;
};

__device__ __forceinline__ int wrap(int s, int n) { return s < 0 ? s + n : (s >= n ? s - n : s); }

// Per-lattice values a tile needs, copied out of the descriptor once.
struct TileConst {
  int n0, n1, n2;
  uint64_t slab_bytes;
  bool w0, w1, w2;
  float lam[3], inv_lam[3], inv_lam2[3], hil[3], mfac[3], anom[3], uref[3], g[3];
  float W[3][3], WW[3][3];
  float omega, coef, inv_scale, scale, om1, oms, one;
  bool mrt;
  float om1g, cdev, ciso, coefb;
};

// Pulled populations of one node in storage format (FP32 value, or the raw
// 16 bits of an FP16 / BF16 value).
template <int S, int Q>
struct Pops {
  typename Store<S>::R v[Q];
  __device__ __forceinline__ float get(int i) const { return Store<S>::to_float(v[i]); }
};

// Byte offsets, within one plane of the marched axis, of the nodes a node
// pulls from (x - c_x, y - c_y) and of the node itself; wall flags mark the
// neighbours that lie beyond a wall. They do not change along the march, so a
// tile computes them once; the plane and the direction enter as a uniform
// base address. Planes hold fewer than 2^30 nodes, so FP32 offsets fit 32 bits.
struct NodeOffs {
  uint32_t o[3][3];  // [c_x + 1][c_y + 1]
  uint32_t own;
  bool ox[3], oy[3];
};

// Buffer resources of the plane slabs a node of plane z pulls from, z - c_z
// for c_z = -1, 0, 1 (so r[1] is plane z itself); oz marks source planes beyond
// a wall. Formed once per plane in uniform control flow and shared by every
// fetch of that plane.
struct PlaneSrc {
  Rsrc r[3];  // [c_z + 1]
  bool oz[3];
};

template <int D, int S, bool WALL>
struct Puller {
  using T = typename Store<S>::T;
  using R = typename Store<S>::R;
  static constexpr int Q = Geo<D, S>::Q;

  __device__ static __forceinline__ void offsets(const TileConst& k, int x, int y, NodeOffs& no) {
    constexpr int sz = sizeof(T);
    int sx[3], sy[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int ax = x - (c - 1), ay = y - (c - 1);
      no.ox[c] = WALL && k.w0 && (ax < 0 || ax >= k.n0);
      no.oy[c] = WALL && k.w1 && (ay < 0 || ay >= k.n1);
      sx[c] = wrap(ax, k.n0);
      sy[c] = (D == 3) ? wrap(ay, k.n1) * k.n0 : 0;
    }
#pragma unroll
    for (int c0 = 0; c0 < 3; ++c0)
#pragma unroll
      for (int c1 = 0; c1 < 3; ++c1) no.o[c0][c1] = uint32_t(sx[c0] + sy[c1]) * sz;
    no.own = uint32_t(x + k.n0 * y) * sz;
  }

  // Issues the loads of the populations arriving at a node of marched plane z
  // from the planes z - c_z; the values land in h in storage format. `sb` is
  // the byte distance of consecutive direction arrays in a slab. Where `near`
  // (uniform: the tile or the plane touches a wall) the halfway bounce-back
  // applies: a population that would arrive from beyond a wall is the node's
  // own post-collision population of the opposite direction.
  __device__ static __forceinline__ void fetch(uint32_t sb, const PlaneSrc& ps, const NodeOffs& no, bool near,
                                               Pops<S, Q>& h) {
    if (WALL && near) {
      // all loads first, then the per-lane choices (a choice right after its
      // own loads would make each direction wait for them in turn)
      R bb[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int c0 = cq<D>(i, 0), c1 = cq<D>(i, 1), c2 = cq<D>(i, 2);
        h.v[i] = Store<S>::load(ps.r[c2 + 1], no.o[c0 + 1][c1 + 1], i * sb);
        bb[i] = i == Q / 2 ? h.v[i] : Store<S>::load(ps.r[1], no.own, (Q - 1 - i) * sb);
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int c0 = cq<D>(i, 0), c1 = cq<D>(i, 1), c2 = cq<D>(i, 2);
        const bool out = (c0 != 0 && no.ox[c0 + 1]) || (c1 != 0 && no.oy[c1 + 1]) || (c2 != 0 && ps.oz[c2 + 1]);
        h.v[i] = out ? bb[i] : h.v[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int c0 = cq<D>(i, 0), c1 = cq<D>(i, 1), c2 = cq<D>(i, 2);
        h.v[i] = Store<S>::load(ps.r[c2 + 1], no.o[c0 + 1][c1 + 1], i * sb);
      }
    }
  }

  // Deviation moments drho = sum h, dj_a = lambda_a sum c_ia h of fetched values.
  __device__ static __forceinline__ void moments(const TileConst& k, const Pops<S, Q>& h, float& drho,
                                                 float (&dj)[3]) {
    float v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = h.get(i);
    float r, m[3];
    line_moments(v, S == 1 ? k.one : 1.f, r, m);
    // values are in storage scale: the factors carry 1/scale
    drho = r * k.inv_scale;
    dj[0] = k.mfac[0] * m[0];
    dj[1] = k.mfac[1] * m[1];
    dj[2] = k.mfac[2] * m[2];
  }

  // Moments of the 3^D values in lattice order: sums along x-lines of three
  // first, then combined (fewer additions than direction by direction).
  // The x-line sums are written as FMAs by `one` (1.0): with FP16 storage the
  // caller passes a 1.0 the compiler cannot see, so each FMA takes its 16-bit
  // operands directly (mixed-precision FMA) instead of converting every value
  // first; a + 1.0 b rounds exactly as a + b, so the sums are unchanged.
  __device__ static __forceinline__ void line_moments(const float (&v)[Q], float one, float& r, float (&m)[3]) {
    if (D == 3) {
      float s[3][3], jx = 0.f;
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2)
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) {
          const int b = 3 * k1 + 9 * k2;
          s[k1][k2] = __builtin_fmaf(v[b + 2], one, __builtin_fmaf(v[b], one, v[b + 1]));
          jx += __builtin_fmaf(v[b], -one, v[b + 2]);
        }
      float rr = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2) rr += (s[0][k2] + s[1][k2]) + s[2][k2];
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2) jy += s[2][k2] - s[0][k2];
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) jz += s[k1][2] - s[k1][0];
      r = rr;
      m[0] = jx;
      m[1] = jy;
      m[2] = jz;
    } else {
      float s[3], jx = 0.f;
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2) {
        const int b = 3 * k2;
        s[k2] = __builtin_fmaf(v[b + 2], one, __builtin_fmaf(v[b], one, v[b + 1]));
        jx += __builtin_fmaf(v[b], -one, v[b + 2]);
      }
      r = (s[0] + s[1]) + s[2];
      m[0] = jx;
      m[1] = 0.f;
      m[2] = s[2] - s[0];
    }
  }
};

// Anomaly Q~_a = j_a (lambda_a^2 - 3T) - j_a u_a^2 of one axis.
__device__ __forceinline__ float anomaly(const TileConst& k, int a, float dja, float ir) {
  const float j = k.uref[a] + dja;
  const float u = j * ir;
  return j * k.anom[a] - j * u * u;
}

// Copies a lattice's per-tile constants out of its descriptor; qbytes = Q
// times the element size.
template <bool WALL>
__device__ __forceinline__ void load_const(const LatticeDesc* __restrict__ Ld, uint32_t qbytes, TileConst& k) {
  k.n0 = Ld->n[0];
  k.n1 = Ld->n[1];
  k.n2 = Ld->n[2];
  k.slab_bytes = uint64_t(Ld->pstride) * qbytes;
  k.w0 = WALL && Ld->wall[0];
  k.w1 = WALL && Ld->wall[1];
  k.w2 = WALL && Ld->wall[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    k.lam[a] = Ld->lam[a];
    k.inv_lam[a] = Ld->inv_lam[a];
    k.inv_lam2[a] = Ld->inv_lam2[a];
    k.hil[a] = Ld->half_inv_lam[a];
    k.mfac[a] = Ld->mfac[a];
    k.anom[a] = Ld->anom[a];
    k.uref[a] = Ld->uref[a];
    k.g[a] = Ld->g[a];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      k.W[a][c] = Ld->W[a][c];
      k.WW[a][c] = Ld->WW[a][c];
    }
  }
  k.omega = Ld->omega;
  k.coef = Ld->coef;
  k.inv_scale = Ld->inv_scale;
  k.scale = Ld->scale;
  k.om1 = Ld->om1;
  k.oms = Ld->oms;
  k.one = Ld->one;
  k.mrt = Ld->mrt != 0;
  k.om1g = Ld->om1g;
  k.cdev = Ld->cdev;
  k.ciso = Ld->ciso;
  k.coefb = Ld->coefb;
}

// Collision of one node (Sec. 2.1, eq. LBGK; Sec. 2.2-2.4): from the
// deviation moments (drho, dj), the central differences of the anomaly Gd
// (already divided by 2 lambda_a) and the pulled values hval(i) (storage
// scale), emits the relaxed and forced populations o_i in storage scale
// through emit(i, o_i).
//
// ACC (FP32 storage) keeps the FP32 rounding error relative to small
// quantities in two places, where 16-bit storage, whose own rounding is
// 2^13 times coarser, gains nothing from it:
// * the velocity deviation x / rho, x = dj - drho u_ref, is formed as
//   x - (x drho) / rho: the rounding of rho = 1 + drho and of its reciprocal
//   then only touches the small correction term (x / rho directly carries a
//   relative error of about one ulp of rho into every velocity, and the
//   relaxation turns a velocity error into a momentum error of about omega
//   times that, every step);
// * the relaxation is applied to the non-equilibrium part,
//   o = e + (1 - w)(h - e) with e = scale (f* - w) and h - e exact while the
//   node is near equilibrium, instead of (1 - w) h + w e, whose two terms
//   nearly cancel when w is close to 2 (one more operation per population).
template <int D, bool FORCE, bool ACC, bool MRT3, class HV, class EMIT>
__device__ __forceinline__ void collide(const TileConst& k, float drho, const float (&dj)[3], const float (&Gd)[3],
                                        HV hval, EMIT emit) {
  constexpr int Q = D == 3 ? 27 : 9;
  const float rho = 1.f + drho;
  const float ir = recip(rho);
  float du[3], dP[3], d[3][3], p[3][3];
  // Multi-relaxation-time collision (a runtime branch for D2Q9, the MRT3
  // kernel variant for D3Q27): the isotropic part of the anomaly difference
  // (its mean over the axes; D2Q9 uses internal axes 0, 2) takes the bulk
  // rate's factor
  const bool mrt = MRT3 || (D == 2 && k.mrt);
  const float giso = !mrt ? 0.f : (D == 3 ? (Gd[0] + Gd[1] + Gd[2]) * (1.f / 3.f) : 0.5f * (Gd[0] + Gd[2]));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (D == 2 && a == 1) {
      du[a] = 0.f;
      dP[a] = 0.f;
    } else {
      const float x = dj[a] - drho * k.uref[a];
      du[a] = ACC ? __builtin_fmaf(-(x * drho), ir, x) : x * ir;
      const float u = k.uref[a] + du[a];
      const float corr = mrt ? k.coef * (Gd[a] - giso) + k.coefb * giso : k.coef * Gd[a];
      dP[a] = du[a] * (u + k.uref[a]) + corr * ir;
    }
    const float t1v = du[a] * k.inv_lam[a];
    const float t2v = dP[a] * k.inv_lam2[a];
    d[a][0] = 0.5f * (t2v - t1v);
    d[a][1] = -t2v;
    d[a][2] = 0.5f * (t2v + t1v);
#pragma unroll
    for (int c = 0; c < 3; ++c) p[a][c] = k.W[a][c] + d[a][c];
  }

  // body force: increments of the equilibrium triplets from u to u + g
  float pe[3][3], e[3][3];
  if (FORCE) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float u = k.uref[a] + du[a];
      const float t1v = du[a] * k.inv_lam[a];
      const float t2v = du[a] * (u + k.uref[a]) * k.inv_lam2[a];
      pe[a][0] = k.W[a][0] + 0.5f * (t2v - t1v);
      pe[a][1] = k.W[a][1] - t2v;
      pe[a][2] = k.W[a][2] + 0.5f * (t2v + t1v);
      const float gg = k.g[a] * (2.f * u + k.g[a]);
      const float s1 = k.g[a] * k.inv_lam[a];
      const float s2 = gg * k.inv_lam2[a];
      e[a][0] = 0.5f * (s2 - s1);
      e[a][1] = -s2;
      e[a][2] = 0.5f * (s2 + s1);
    }
  }

  // Relaxation (Sec. 2.1, eq. LBGK) in storage scale,
  //   o_i = (1 - w) h_i + w scale (f*_i - w_i) (+ scale F_i),
  // with f*_i - w_i = drho B_i + dB_i from the product deviation. The
  // factor m = w scale (ACC: m = scale, the relaxation follows) and the
  // (c_x, c_y) partial products are applied once per node:
  // m (drho X + dX) p_z + W_x W_y (m d_z) for D3Q27,
  // m (drho W~_x + d_x) p_y + W_x (m d_y) for D2Q9.
  const float mfold = (ACC || MRT3) ? k.scale : k.oms;
  const float drs = mfold * drho;
  float ds[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) ds[a][c] = mfold * d[a][c];
  float A[3][3];  // [c_x][c_y]; D2Q9 uses [c_x][1]
#pragma unroll
  for (int c0 = 0; c0 < 3; ++c0)
#pragma unroll
    for (int c1 = 0; c1 < 3; ++c1) {
      if (D == 3) {
        const float X = p[0][c0] * p[1][c1];
        const float dXs = ds[0][c0] * p[1][c1] + k.W[0][c0] * ds[1][c1];
        A[c0][c1] = drs * X + dXs;
      } else if (c1 == 1) {
        A[c0][c1] = drs * p[0][c0] + ds[0][c0];
      }
    }
  // Force F_i = rho (prod (pe + e) - prod pe) in storage scale, with the
  // factor scale rho folded into the x-axis triplets once per node:
  // F_i scale = dY (pe_z + e_z) + Y e_z, Y = sx_x pe_y, dY = ex_x (pe_y + e_y) + sx_x e_y,
  // sx = scale rho pe_x, ex = scale rho e_x (D2Q9: pe_y = 1, e_y = 0).
  float sx[3], ex[3], qz[3];
  if (FORCE) {
    const float sr = k.scale * rho;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sx[c] = sr * pe[0][c];
      ex[c] = sr * e[0][c];
      qz[c] = pe[2][c] + e[2][c];
    }
  }
  if constexpr (D == 3 && MRT3) {
    // Multi-relaxation-time relaxation in storage scale (as the D2Q9 branch
    // below, over three axes): fe_i = scale (f*_i - w_i) = A p_z + W_x W_y ds_z
    // with m = scale, n_i = h_i - fe_i, and
    //   o_i = fe_i + (1 - og) n_i + (og - o) G_i(Pi_dev) + (og - ob) G_i(Pi_iso),
    // G_i(Pi) = sum_a dPsi_a/dP Pi_aa prod_{b != a} p_b
    //         + sum_{a<b} c_a c_b Pi_ab / (4 lam_a lam_b) p_d   (d the third axis).
    // The second moments of n are those of h less those of fe, which the
    // product form gives in closed form: sum c_a^2 f* = rho (p_a+ + p_a-),
    // sum c_a c_b f* = rho (p_a+ - p_a-)(p_b+ - p_b-), and the same of w with
    // the reference triplets W (written in deviations: rho = 1 + drho,
    // p = W + d), so no fe_i is formed before the emitting pass.
    float s2[3] = {0.f, 0.f, 0.f}, s11[3] = {0.f, 0.f, 0.f};  // sum c_a^2 h; sum c_x c_y h, c_x c_z h, c_y c_z h
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const int c0 = cq<3>(i, 0), c1 = cq<3>(i, 1), c2 = cq<3>(i, 2);
      const float hv = hval(i);
      if (c0 != 0) s2[0] += hv;
      if (c1 != 0) s2[1] += hv;
      if (c2 != 0) s2[2] += hv;
      if (c0 * c1 > 0) s11[0] += hv;
      if (c0 * c1 < 0) s11[0] -= hv;
      if (c0 * c2 > 0) s11[1] += hv;
      if (c0 * c2 < 0) s11[1] -= hv;
      if (c1 * c2 > 0) s11[2] += hv;
      if (c1 * c2 < 0) s11[2] -= hv;
    }
    const float sc = k.scale;
    float pd[3], U[3], dl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float e2 = sc * (drho * (k.W[a][0] + k.W[a][2]) + rho * (d[a][0] + d[a][2]));
      pd[a] = (s2[a] - e2) * (k.lam[a] * k.lam[a]);
      U[a] = k.W[a][2] - k.W[a][0];  // u_ref / lam
      dl[a] = d[a][2] - d[a][0];     // du / lam
    }
    auto e11 = [&](int a, int b) {
      return sc * (drho * U[a] * U[b] + rho * (U[a] * dl[b] + dl[a] * U[b] + dl[a] * dl[b]));
    };
    const float qxy = 0.25f * (s11[0] - e11(0, 1)), qxz = 0.25f * (s11[1] - e11(0, 2));
    const float qyz = 0.25f * (s11[2] - e11(1, 2));
    const float tr = (pd[0] + pd[1] + pd[2]) * (1.f / 3.f);
    const float dv0 = pd[0] - tr, dv1 = pd[1] - tr, dv2 = pd[2] - tr;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const int c0 = cq<3>(i, 0) + 1, c1 = cq<3>(i, 1) + 1, c2 = cq<3>(i, 2) + 1;
      const float fe = A[c0][c1] * p[2][c2] + k.WW[c0][c1] * ds[2][c2];
      const float nq = hval(i) - fe;
      const float gx = c0 == 1 ? -k.inv_lam2[0] : 0.5f * k.inv_lam2[0];
      const float gy = c1 == 1 ? -k.inv_lam2[1] : 0.5f * k.inv_lam2[1];
      const float gz = c2 == 1 ? -k.inv_lam2[2] : 0.5f * k.inv_lam2[2];
      const float px = p[0][c0], py = p[1][c1], pz = p[2][c2];
      const float tx = gx * py * pz, ty = px * gy * pz, tz = px * py * gz;
      const float gdev = tx * dv0 + ty * dv1 + tz * dv2 + float((c0 - 1) * (c1 - 1)) * qxy * pz +
                         float((c0 - 1) * (c2 - 1)) * qxz * py + float((c1 - 1) * (c2 - 1)) * qyz * px;
      const float gis = (tx + ty + tz) * tr;
      float o = fe + k.om1g * nq + k.cdev * gdev + k.ciso * gis;
      if (FORCE) {
        const float Y = sx[c0] * pe[1][c1];
        const float dY = ex[c0] * (pe[1][c1] + e[1][c1]) + sx[c0] * e[1][c1];
        o += dY * qz[c2] + Y * e[2][c2];
      }
      emit(i, o);
    }
    return;
  }
  if constexpr (D == 2) {
    if (mrt) {
      // Multi-relaxation-time relaxation in storage scale: fe_i = scale
      // (f*_i - w_i), n_i = h_i - fe_i; the non-equilibrium stress (physical
      // x = internal 0, y = internal 2) relaxes at omega (deviator) and
      // omega_bulk (trace), the rest at omega_ghost:
      //   o_i = fe_i + (1 - og) n_i + (og - o) G_i(Pi_dev) + (og - ob) G_i(Pi_iso),
      // G the linear Grad map at the collision's triplets p (dPsi/dP = -1/lam^2
      // at c = 0, 1/(2 lam^2) at c = +-1; c_x c_y Pi_xy / (4 lam_x lam_y)).
      const float sc = k.scale, scr = sc * drho;
      // two passes that recompute fe_i rather than hold it (register budget
      // of the LBGK path, which shares this kernel)
      auto feq = [&](int cx, int cy) {
        return (scr * p[0][cx + 1] + sc * d[0][cx + 1]) * p[2][cy + 1] + k.W[0][cx + 1] * (sc * d[2][cy + 1]);
      };
      float pxx = 0.f, pyy = 0.f, pxy = 0.f;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int cx = cq<2>(i, 0), cy = cq<2>(i, 2);
        const float nq = hval(i) - feq(cx, cy);
        if (cx != 0) pxx += nq;
        if (cy != 0) pyy += nq;
        if (cx * cy > 0) pxy += nq;
        if (cx * cy < 0) pxy -= nq;
      }
      pxx *= k.lam[0] * k.lam[0];
      pyy *= k.lam[2] * k.lam[2];
      const float dev = 0.5f * (pxx - pyy), iso = 0.5f * (pxx + pyy);
      const float qxy = pxy * 0.25f;  // lam_x lam_y Pi_xy-sum / (4 lam_x lam_y)
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int cx = cq<2>(i, 0), cy = cq<2>(i, 2);
        const float fe = feq(cx, cy);
        const float nq = hval(i) - fe;
        const float gx = cx == 0 ? -k.inv_lam2[0] : 0.5f * k.inv_lam2[0];
        const float gy = cy == 0 ? -k.inv_lam2[2] : 0.5f * k.inv_lam2[2];
        const float px = p[0][cx + 1], py = p[2][cy + 1];
        const float gdev = (gx * py - px * gy) * dev + float(cx * cy) * qxy;
        const float gis = (gx * py + px * gy) * iso;
        float o = fe + k.om1g * nq + k.cdev * gdev + k.ciso * gis;
        if (FORCE) o += ex[cx + 1] * qz[cy + 1] + sx[cx + 1] * e[2][cy + 1];
        emit(i, o);
      }
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int c0 = cq<D>(i, 0) + 1, c1 = cq<D>(i, 1) + 1, c2 = cq<D>(i, 2) + 1;
    const float Wc = D == 3 ? k.WW[c0][c1] : k.W[0][c0];
    const float fe = A[c0][c1] * p[2][c2] + Wc * ds[2][c2];
    float o = ACC ? 0.f : fe;
    if (FORCE) {
      if (D == 3) {
        const float Y = sx[c0] * pe[1][c1];
        const float dY = ex[c0] * (pe[1][c1] + e[1][c1]) + sx[c0] * e[1][c1];
        o += dY * qz[c2] + Y * e[2][c2];
      } else {
        o += ex[c0] * qz[c2] + sx[c0] * e[2][c2];
      }
    }
    if (ACC) {
      const float hv = hval(i);
      emit(i, __builtin_fmaf(k.om1, hv - fe, fe) + o);
    } else {
      emit(i, k.om1 * hval(i) + o);
    }
  }
}

// ---- diagnostics folded into a step ----
// A node's record contribution is kDF FP64 values, in this order: mass, the
// three momentum components, |u|^2, the mode's real and imaginary parts, the
// mode's max |amplitude| (max), the least density (min) and the count of
// non-finite nodes. Plane by plane, each 16-lane row of a wave folds its
// nodes' values with DPP lane permutations, and lane (row r, field j) adds the
// row's value of field j into LDS slot (wave, r, j); the block's partial
// record is the fold of its slots in (wave, row) order. Every step of this is
// fixed, so a record is reproducible bitwise for a given launch grid.
constexpr int kDF = 10;
constexpr int kDiagRows = 4;  // 16-lane rows per wave
__device__ __forceinline__ constexpr int diag_kind(int j) { return j == 7 ? 1 : (j == 8 ? 2 : 0); }
__device__ __forceinline__ constexpr double diag_identity(int j) { return j == 8 ? 1e300 : 0.0; }
__device__ __forceinline__ double diag_op(int kind, double x, double y) {
  return kind == 0 ? x + y : (kind == 1 ? fmax(x, y) : fmin(x, y));
}
// record field of accumulated value j
__device__ __forceinline__ constexpr int diag_rec_field(int j) { return j + 1 + (j >= 5 ? 1 : 0); }

// x of another lane of the same 16-lane row (DPP control CTRL), both halves
template <int CTRL>
__device__ __forceinline__ double dpp64(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int l2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  const int h2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(h2, l2);
}

// One node's contribution c[] from its pulled values hval(i) (storage scale):
// rho and the reported velocity u = j/rho + g/2 in FP64; u is also staged in
// FP32 for the enstrophy pass. (x0, x1, x2) are the node's internal indices
// and cell its index with x fastest; internal axis a is physical axis a for
// D3Q27, and 0 -> x, 2 -> y for D2Q9.
// The node's value of field j goes to put(j, value) as soon as it is formed.
template <int D, class HV, class PUT>
__device__ __forceinline__ void diag_node(const DiagArgs& da, HV hval, int x0, int x1, int x2, int64_t cell,
                                          PUT put) {
  constexpr int Q = D == 3 ? 27 : 9;
  double r = 0.0, m[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double v = double(hval(i));
    r += v;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ci = cq<D>(i, a);
      if (ci > 0) m[a] += v;
      if (ci < 0) m[a] -= v;
    }
  }
  const double mp[3] = {m[0], D == 3 ? m[1] : m[2], D == 3 ? m[2] : 0.0};
  const double rho = 1.0 + r * da.inv_scale;
  const double ir = 1.0 / rho;
  double u[3];
  bool finite = isfinite(rho);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = (a < D) ? (da.uref[a] + da.lam[a] * mp[a] * da.inv_scale) * ir + 0.5 * da.g[a] : 0.0;
    finite = finite && isfinite(u[a]);
    da.ustage[a * da.N + cell] = float(u[a]);
  }
  put(0, rho);
  put(1, rho * u[0]);
  put(2, rho * u[1]);
  put(3, rho * u[2]);
  put(4, u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  put(8, finite ? rho : -1e300);
  put(9, finite ? 0.0 : 1.0);
  double mre = 0.0, mim = 0.0, mabs = 0.0;
  if (da.has_mode) {
    // e^{i k.x} as the product of the per-axis factors e^{i k_a lam_a x_a}
    const int xp[3] = {x0, D == 3 ? x1 : x2, D == 3 ? x2 : 0};
    const double* e = da.mode_tab + 2 * (da.mode_off[0] + xp[0]);
    double cs = e[0], sn = e[1];
#pragma unroll
    for (int a = 1; a < D; ++a) {
      e = da.mode_tab + 2 * (da.mode_off[a] + xp[a]);
      const double ca = e[0], sa = e[1];
      const double c2 = cs * ca - sn * sa;
      sn = sn * ca + cs * sa;
      cs = c2;
    }
    const double up = da.mode_dir[0] * u[0] + da.mode_dir[1] * u[1] + da.mode_dir[2] * u[2];
    mre = up * cs;
    mim = -up * sn;
    mabs = fabs(up);
  }
  put(5, mre);
  put(6, mim);
  put(7, mabs);
}

__device__ __forceinline__ void diag_clear(double (&c)[kDF]) {
#pragma unroll
  for (int j = 0; j < kDF; ++j) c[j] = diag_identity(j);
}

// Row fold of one field's value (see diag_wave_fold), and its store by the
// lanes jl == j: for a caller with the whole wave active.
__device__ __forceinline__ void diag_fold_one(int j, double x, double* __restrict__ wslot) {
  const int kind = diag_kind(j);
  x = diag_op(kind, x, dpp64<0xB1>(x));
  x = diag_op(kind, x, dpp64<0x4E>(x));
  x = diag_op(kind, x, dpp64<0x141>(x));
  x = diag_op(kind, x, dpp64<0x140>(x));
  const int lane = threadIdx.x & 63;
  if ((lane & 15) == j) wslot[(lane >> 4) * kDF + j] = diag_op(kind, wslot[(lane >> 4) * kDF + j], x);
}

// Row fold of c[] (lanes i and i^1, i^2, then the mirrored lanes of each
// half row and of the row: each pairwise operation is commutative, so all
// 16 lanes of a row end with the same values), then lane (r, j) adds the
// row's field j into wslot[r kDF + j]. Called by every lane of the wave.
__device__ __forceinline__ void diag_wave_fold(double (&c)[kDF], double* __restrict__ wslot) {
#pragma unroll
  for (int j = 0; j < kDF; ++j) {
    const int kind = diag_kind(j);
    double x = c[j];
    x = diag_op(kind, x, dpp64<0xB1>(x));   // quad_perm [1,0,3,2]
    x = diag_op(kind, x, dpp64<0x4E>(x));   // quad_perm [2,3,0,1]
    x = diag_op(kind, x, dpp64<0x141>(x));  // row_half_mirror
    x = diag_op(kind, x, dpp64<0x140>(x));  // row_mirror
    c[j] = x;
  }
  const int lane = threadIdx.x & 63, jl = lane & 15, r = lane >> 4;
  double v = c[0];
  int kind = 0;
#pragma unroll
  for (int j = 1; j < kDF; ++j) {
    v = jl == j ? c[j] : v;
    kind = jl == j ? diag_kind(j) : kind;
  }
  if (jl < kDF) wslot[r * kDF + jl] = diag_op(kind, wslot[r * kDF + jl], v);
}

__device__ __forceinline__ void diag_slots_init(double* __restrict__ wslot) {
  const int lane = threadIdx.x & 63, jl = lane & 15, r = lane >> 4;
  if (jl < kDF) wslot[r * kDF + jl] = jl == 8 ? 1e300 : 0.0;
}

// The block's partial record from its slots, folded in (wave, row) order.
template <int NW>
__device__ __forceinline__ void diag_block_store(const double* __restrict__ wsum, double* __restrict__ partials) {
  __syncthreads();
  const int j = threadIdx.x;
  if (j < kDF) {
    const int kind = j == 7 ? 1 : (j == 8 ? 2 : 0);
    double r = wsum[j];
    for (int k = 1; k < NW * kDiagRows; ++k) r = diag_op(kind, r, wsum[k * kDF + j]);
    partials[blockIdx.x * kRec + (j + 1 + (j >= 5 ? 1 : 0))] = r;
  }
  if (j == kDF) partials[blockIdx.x * kRec + R_STEP] = 0.0;
}

template <int D, int S, bool WALL, bool FORCE, bool DIAG, bool MRT3>
__device__ __forceinline__ void step_tile(const LatticeDesc* __restrict__ Ld, int64_t tl, int parity,
                                          float* __restrict__ sq, const DiagArgs& da, double* __restrict__ wslot) {
  using G = Geo<D, S>;
  using T = typename Store<S>::T;
  using P = Puller<D, S, WALL>;
  constexpr int Q = G::Q, TXW = G::TXW, TYR = G::TYR;

  TileConst k;
  load_const<WALL>(Ld, Q * sizeof(T), k);
  const char* src = static_cast<const char*>(Ld->buf[parity]);
  const char* dst = static_cast<const char*>(Ld->buf[parity ^ 1]);

  const int tiles0 = Ld->tiles[0], tiles1 = Ld->tiles[1], chunk = Ld->chunk;
  const int t0 = int(tl % tiles0);
  const int64_t rr = tl / tiles0;
  const int t1 = int(rr % tiles1);
  const int t2 = int(rr / tiles1);
  const int x0 = t0 * TXW, y0 = t1 * TYR;
  const int z0 = t2 * chunk;
  const int z1 = min(z0 + chunk, k.n2);
  // Odd chunks march down the axis: the ring planes at the face between two
  // chunks are then read by both tiles at about the same time (both early or
  // both late in the step), so the second read is a cache hit instead of an
  // HBM read. Reversing the march changes no result: the z difference takes
  // the sign of the march, and every operation is otherwise the same.
  const int dir = (t2 & 1) ? -1 : 1;
  const int zs = dir > 0 ? z0 : z1 - 1, len = z1 - z0;
  const int xe = min(x0 + TXW, k.n0), ye = min(y0 + TYR, k.n1);

  const int tid = threadIdx.x;
  const int lx = D == 3 ? (tid & 63) : tid;
  const int ly = D == 3 ? (tid >> 6) : 0;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool active = gx < k.n0 && gy < k.n1;

  // anomaly exchange in LDS, double buffered by plane: axis 0 at
  // sq[b LX + slot], axis 1 at sq[2 LX + b LY + slot] (plain indices into the
  // shared array keep every access an LDS instruction)
  auto QX = [&](int b, int slot) -> float& { return sq[b * G::LX + slot]; };
  auto QY = [&](int b, int slot) -> float& { return sq[2 * G::LX + b * G::LY + slot]; };

  // ---- neighbour slots of the tiled axes (fixed over the march) ----
  const int rowx = ly * (TXW + 2);
  const int sx_own = rowx + lx + 1;
  bool gxm = false, gxp = false, gym = false, gyp = false;  // neighbour is a wall ghost
  int sxm, sxp, sym = 0, syp = 0, sy_own = 0;
  {
    int xm = gx - 1, xp = gx + 1;
    if (gx == 0) { if (k.w0) gxm = true; else xm = k.n0 - 1; }
    if (gx == k.n0 - 1) { if (k.w0) gxp = true; else xp = 0; }
    sxm = (xm >= x0 && xm < xe) ? rowx + (xm - x0) + 1 : rowx;
    sxp = (xp >= x0 && xp < xe) ? rowx + (xp - x0) + 1 : rowx + TXW + 1;
    if (D == 3) {
      int ym = gy - 1, yp = gy + 1;
      if (gy == 0) { if (k.w1) gym = true; else ym = k.n1 - 1; }
      if (gy == k.n1 - 1) { if (k.w1) gyp = true; else yp = 0; }
      sy_own = (ly + 1) * TXW + lx;
      sym = (ym >= y0 && ym < ye) ? (ym - y0 + 1) * TXW + lx : lx;
      syp = (yp >= y0 && yp < ye) ? (yp - y0 + 1) * TXW + lx : (TYR + 1) * TXW + lx;
    }
  }

  // ---- halo node served by this thread (if any) ----
  bool has_halo = false;
  int hx = 0, hy = 0, hax = 0, hslot = 0;
  if (tid < G::HY) {
    const int side = tid / TXW, col = tid % TXW;
    hx = x0 + col;
    hax = 1;
    hslot = (side ? (TYR + 1) * TXW : 0) + col;
    has_halo = hx < k.n0;
    if (side == 0) {
      hy = y0 - 1;
      if (y0 == 0) { if (k.w1) has_halo = false; else hy = k.n1 - 1; }
    } else {
      hy = y0 + TYR;
      if (hy >= k.n1) { if (k.w1) has_halo = false; else hy = 0; }
    }
  } else if (tid < G::HY + G::HX) {
    const int q = tid - G::HY;
    const int side = q / TYR, row = q % TYR;
    hy = y0 + row;
    hax = 0;
    hslot = row * (TXW + 2) + (side ? TXW + 1 : 0);
    has_halo = hy < k.n1;
    if (side == 0) {
      hx = x0 - 1;
      if (x0 == 0) { if (k.w0) has_halo = false; else hx = k.n0 - 1; }
    } else {
      hx = x0 + TXW;
      if (hx >= k.n0) { if (k.w0) has_halo = false; else hx = 0; }
    }
  }
  const int hofs = hax == 0 ? 0 : 2 * G::LX;     // buffer 0 of the halo's axis
  const int hstep = hax == 0 ? G::LX : G::LY;    // offset to buffer 1

  // the halo node's axis is a run-time value: select its constants once
  const float h_uref = hax == 0 ? k.uref[0] : k.uref[1];
  const float h_anom = hax == 0 ? k.anom[0] : k.anom[1];
  NodeOffs hno;
  P::offsets(k, hx, hy, hno);
  // anomaly of the halo node from its fetched populations, into LDS buffer b
  auto halo_store = [&](const Pops<S, Q>& hv, int b) {
    float dr, dj[3];
    P::moments(k, hv, dr, dj);
    const float ir = recip(1.f + dr);
    const float j = h_uref + (hax == 0 ? dj[0] : dj[1]);
    const float u = j * ir;
    sq[hofs + b * hstep + hslot] = j * h_anom - j * u * u;
  };
  // Plane index along the marched axis, reduced into the lattice: beyond it
  // the index wraps (periodic axis) or, behind a wall, the plane is a ghost
  // and the returned index is only a valid stand-in.
  auto plane = [&](int zz, bool& ghost) {
    ghost = false;
    if (zz < 0) {
      if (k.w2) ghost = true;
      zz += k.n2;
    }
    while (zz >= k.n2) {
      if (k.w2) ghost = true;
      zz -= k.n2;
    }
    return zz;
  };

  auto src_planes = [&](int zz) {
    PlaneSrc ps;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int az = zz - (c - 1);
      ps.oz[c] = WALL && k.w2 && (az < 0 || az >= k.n2);
      ps.r[c] = rsrc(src + uint64_t(wrap(az, k.n2)) * k.slab_bytes);
    }
    return ps;
  };
  const int cx = active ? gx : 0, cy = active ? gy : 0;
  NodeOffs no;
  P::offsets(k, cx, cy, no);
  // A wave takes the bounce-back fetch path (uniform) only if one of its
  // lanes' nodes, resp. halo nodes, pulls from beyond a wall of a tiled axis,
  // or the plane from beyond a wall of the marched axis; in a tile next to a
  // y wall that is the wave of the wall row (and the x-halo lanes), not the
  // whole tile.
  auto beyond = [](const NodeOffs& o) { return o.ox[0] || o.ox[2] || o.oy[0] || o.oy[2]; };
  const bool near_own = WALL && __ballot(beyond(no)) != 0;
  const bool near_halo = WALL && __ballot(has_halo && beyond(hno)) != 0;
  auto near = [&](const PlaneSrc& ps, bool xy) { return xy || ps.oz[0] || ps.oz[2]; };
  const uint32_t sb0 = uint32_t(Ld->pstride) * uint32_t(sizeof(T));

  // Populations in flight: while plane z is relaxed one set holds plane z,
  // one the next plane in march order (fetched a plane ahead) and one receives
  // the plane after it; hp holds the halo node's next plane.
  Pops<S, Q> P0, P1, P2, hp;
  float drho = 0.f, dj[3] = {0.f, 0.f, 0.f};
  float qc[3] = {0.f, 0.f, 0.f};  // anomaly of the current plane at this node
  float qprev = 0.f;
  // ---- prologue: plane before the chunk (ring), the first plane, and the
  // fetches of the second ----
  {
    bool ghost_prev;
    const int zp = plane(zs - dir, ghost_prev);
    {
      float dr, djp[3];
      const PlaneSrc sp = src_planes(zp);
      P::fetch(sb0, sp, no, near(sp, near_own), P2);
      P::moments(k, P2, dr, djp);
      qprev = anomaly(k, 2, djp[2], recip(1.f + dr));
    }
    const PlaneSrc s0 = src_planes(zs);
    P::fetch(sb0, s0, no, near(s0, near_own), P0);
    P::moments(k, P0, drho, dj);
    {
      const float ir = recip(1.f + drho);
      qc[0] = anomaly(k, 0, dj[0], ir);
      if (D == 3) qc[1] = anomaly(k, 1, dj[1], ir);
      qc[2] = anomaly(k, 2, dj[2], ir);
      if (ghost_prev) qprev = -qc[2];
      if (active) {
        QX(0, sx_own) = qc[0];
        if (D == 3) QY(0, sy_own) = qc[1];
      }
    }
    bool ghost1;
    const PlaneSrc s1 = src_planes(plane(zs + dir, ghost1));
    P::fetch(sb0, s1, no, near(s1, near_own), P1);
    if (has_halo) {
      P::fetch(sb0, s0, hno, near(s0, near_halo), hp);
      halo_store(hp, 0);
      P::fetch(sb0, s1, hno, near(s1, near_halo), hp);
    }
  }
  __syncthreads();

  // One plane of the march. The three population sets rotate roles from
  // plane to plane (the loop below is unrolled by three), so that no register
  // receiving a fetch is ever copied before its load has landed.
  const float hz = dir > 0 ? k.hil[2] : -k.hil[2];  // z difference in march order
  auto march = [&](int m, const Pops<S, Q>& h, const Pops<S, Q>& pf1, Pops<S, Q>& pf2) {
    const int z = zs + dir * m;
    const int b = m & 1;
    // The array distance is made opaque per plane so that the per-direction
    // offsets are formed in scalar registers where they are used rather than
    // held across the march.
    uint32_t sb = sb0;
    asm("" : "+s"(sb) : "s"(z));
    const bool more = m + 1 < len;
    bool ghost_next, ghost2;
    plane(z + dir, ghost_next);
    const PlaneSrc s2 = src_planes(plane(z + 2 * dir, ghost2));
    // The fetches and the moments below are issued by every lane (lanes
    // beyond a ragged edge work on a clamped node; behind a wall the fetched
    // plane goes unused), so that the code between a fetch and its use is
    // straight-line and the waits for the loads count exactly the memory
    // operations issued after them. Fetches of planes the tile never uses are
    // skipped as a whole (a uniform test): the node's plane two on past the
    // ring plane, the halo's plane two on past the last relaxed plane. The node's own
    // fetch precedes the halo's, whose branch then reuses its offsets.
    // next plane (always needed: its anomaly closes the ring)
    float drn, djn[3], qn[3] = {0.f, 0.f, 0.f};
    {
      P::moments(k, pf1, drn, djn);
      const float ir = recip(1.f + drn);
      qn[0] = anomaly(k, 0, djn[0], ir);
      if (D == 3) qn[1] = anomaly(k, 1, djn[1], ir);
      qn[2] = anomaly(k, 2, djn[2], ir);
    }
    if (m + 2 <= len) P::fetch(sb, s2, no, near(s2, near_own), pf2);
    // Memory drains (here, before the collision and after its stores): with
    // the next planes' reads left in flight, the halo and ring rows that
    // neighbouring tiles re-read drop out of L2 (about 18% more HBM reads
    // than the algorithmic bytes at 256^3 FP32, against 6% with the drains,
    // and 6% longer steps).
    drain_vm();
    // halo of the next plane (fetched one plane ahead), then the fetch two planes on
    if (has_halo) {
      halo_store(hp, b ^ 1);
      if (m + 2 < len) P::fetch(sb, s2, hno, near(s2, near_halo), hp);
    }
    const float qnext = ghost_next ? -qc[2] : qn[2];

    double dc[DIAG ? kDF : 1];
    if constexpr (DIAG) diag_clear(dc);
    if (active) {
      // ---- collision of plane z ----
      drain_all();
      const float qxm = gxm ? -qc[0] : QX(b, sxm);
      const float qxp = gxp ? -qc[0] : QX(b, sxp);
      float Gd[3];
      Gd[0] = (qxp - qxm) * k.hil[0];
      Gd[1] = 0.f;
      if (D == 3) {
        const float qym = gym ? -qc[1] : QY(b, sym);
        const float qyp = gyp ? -qc[1] : QY(b, syp);
        Gd[1] = (qyp - qym) * k.hil[1];
      }
      Gd[2] = (qnext - qprev) * hz;

      const Rsrc rd = rsrc(dst + uint64_t(z) * k.slab_bytes);
      collide<D, FORCE, S == 0, MRT3>(k, drho, dj, Gd, [&](int i) { return h.get(i); },
                        [&](int i, float o) { Store<S>::store(rd, no.own, i * sb, o); });
      if constexpr (DIAG)
        diag_node<D>(da, [&](int i) { return h.get(i); }, gx, gy, z,
                     int64_t(gx) + int64_t(k.n0) * (int64_t(gy) + int64_t(k.n1) * z),
                     [&](int j, double v) { dc[j] = v; });
    }
    if constexpr (DIAG) diag_wave_fold(dc, wslot);
    drain_vm();

    if (more && active) {
      QX(b ^ 1, sx_own) = qn[0];
      if (D == 3) QY(b ^ 1, sy_own) = qn[1];
    }
    __syncthreads();
    drho = drn;
    dj[0] = djn[0];
    dj[1] = djn[1];
    dj[2] = djn[2];
    qprev = qc[2];
    qc[0] = qn[0];
    qc[1] = qn[1];
    qc[2] = qnext;
  };
  for (int m = 0; m < len; m += 3) {
    march(m, P0, P1, P2);
    if (m + 1 < len) march(m + 1, P1, P2, P0);
    if (m + 2 < len) march(m + 2, P2, P0, P1);
  }
}

// ---------------------------------------------------------------------------
// LDS-staged D3Q27 step for 16-bit storage.
//
// The kernel above holds two of its three planes' populations in registers,
// which caps it at two waves per SIMD; with 2-byte elements that occupancy,
// rather than HBM, sets its pace. Here a block of 64 x TY nodes stages, for
// every direction i, the rows of plane z - c_iz that its tile and halo nodes
// pull direction i from, in LDS, with direct buffer-to-LDS loads (no
// registers in between): a row's 64 interior nodes in 16-byte pieces, and the
// node pairs left and right of the tile in 4-byte pieces. A pull is then an
// LDS read at an offset fixed per direction. Two planes are staged: the next
// plane in march order, whose values give its anomaly (and are kept in
// registers, two per register, for its relaxation one plane later), and the
// plane after it, whose loads fly while the current plane is relaxed. One
// barrier per plane separates a stage's reads from its reloading.
// It applies to D3Q27 lattices whose n_x is a multiple of 64, x and z
// periodic, and y either bounce-back with n_y a multiple of TY or periodic
// with n_y > TY / 2 (so that every staged row, y0 - 2 ... y0 + TY + 1, lies
// within one period of the axis); the others take the kernel above. On a
// periodic y axis whose n_y is not a multiple of TY the last tile row
// overhangs it: its rows at and beyond n_y hold the wrapped rows 0, 1, ...
// (staged like any other) and give the anomaly that the last real row takes
// as its neighbour's; their stores are dropped.
//
// Stage layout (bytes): 27 boxes of BOX bytes, direction i's at i BOX. Box
// row r (0 ... TY + 1) holds lattice row y0 - 1 - c_iy + r, so a node of tile
// row ly reads row ly + 1 of every box: the 64 interior nodes x0 ... x0 + 63
// at r 128, and, after the TY + 2 interior rows, the pairs x0 - 2, x0 - 1
// and x0 + 64, x0 + 65 of each row at SIDE + 8 r and SIDE + 8 r + 4. A direct
// load writes 16 (or 4) bytes per lane to consecutive LDS addresses from a
// per-instruction base, so each box is written by three instructions of
// 16-byte pieces (eight rows each) and one of 4-byte side pieces.
// ---------------------------------------------------------------------------
namespace lds {
constexpr int TX = 64, TY = kRowsStaged, NT = TX * TY, NW = NT / 64;
constexpr int ROWS = TY + 2;                    // box rows
constexpr int SIDE = ROWS * 128;                // side pairs of a box
constexpr int BOX = SIDE + ROWS * 8;
constexpr int STAGE = 27 * BOX;
constexpr int LXF = TY * (TX + 2);              // anomaly exchange, axis 0 (floats per buffer)
constexpr int LYF = (TY + 2) * TX;              // anomaly exchange, axis 1
constexpr int BYTES = 2 * STAGE + 2 * (LXF + LYF) * 4;
constexpr int IITEMS = ROWS * 8;                // 16-byte pieces of a box
constexpr int IINSTR = (IITEMS + 63) / 64;      // wave instructions for them
constexpr int SITEMS = ROWS * 2;                // 4-byte side pieces of a box
constexpr int PER_BOX = IINSTR + 1;            // wave instructions per box
static_assert(SITEMS <= 64, "one wave instruction stages the side pairs of a box");
static_assert(BOX % 16 == 0 && STAGE % 16 == 0, "16-byte aligned stage destinations");
static_assert(BYTES <= 160 * 1024, "LDS of one block");
static_assert(NT <= 1024 && NT % 64 == 0 && TY % 2 == 0, "one block per tile");
}  // namespace lds

using lds_ptr = __attribute__((address_space(3))) unsigned char*;

// Byte of staged column dx = x - x0 (dx in [-2, 65]) of box row r.
__device__ __forceinline__ int col_byte(int dx, int r) {
  using namespace lds;
  return dx < 0 ? SIDE + 8 * r + 2 * (dx + 2) : (dx < 64 ? 128 * r + 2 * dx : SIDE + 8 * r + 4 + 2 * (dx - 64));
}

// The 27 values of a node, two 16-bit values per register (value i in half
// i & 1 of word i / 2).
struct Held {
  uint32_t w[14];
  __device__ __forceinline__ unsigned short get(int i) const {
    return (i & 1) ? static_cast<unsigned short>(w[i >> 1] >> 16) : static_cast<unsigned short>(w[i >> 1]);
  }
};

// WALLY: halfway bounce-back walls on y (x and z periodic). Rows beyond a wall
// are staged like any other (their values go unused); a node of a row next to
// a wall takes the populations that would arrive through it from its own
// post-collision populations of the opposite directions, loaded directly, and
// the anomaly beyond the wall is the odd ghost -Q~ of the wall row.
template <int S, bool FORCE, bool WALLY, bool DIAG, bool OVER>
__device__ __forceinline__ void step_tile_lds(const LatticeDesc* __restrict__ Ld, int64_t tl, int parity,
                                              unsigned char* __restrict__ smem, const DiagArgs& da,
                                              double* __restrict__ wslot) {
  using namespace lds;
  using T = typename Store<S>::T;
  using R = typename Store<S>::R;
  static_assert(sizeof(T) == 2, "16-bit storage only");
  constexpr int Q = 27;

  TileConst k;
  load_const<WALLY>(Ld, Q * sizeof(T), k);
  const char* src = static_cast<const char*>(Ld->buf[parity]);
  const char* dst = static_cast<const char*>(Ld->buf[parity ^ 1]);
  const uint32_t sb0 = uint32_t(Ld->pstride) * 2u;

  const int tiles0 = Ld->tiles[0], tiles1 = Ld->tiles[1], chunk = Ld->chunk;
  const int t0 = int(tl % tiles0);
  const int64_t rr = tl / tiles0;
  const int t1 = int(rr % tiles1);
  const int t2 = int(rr / tiles1);
  const int x0 = t0 * TX, y0 = t1 * TY;
  const int z0 = t2 * chunk;
  const int z1 = min(z0 + chunk, k.n2);
  // odd chunks march down the axis (see the kernel above)
  const int dir = (t2 & 1) ? -1 : 1;
  const int zs = dir > 0 ? z0 : z1 - 1, len = z1 - z0;

  const int tid = threadIdx.x;
  const int lx = tid & 63, ly = tid >> 6;
  const int gx = x0 + lx, gy = y0 + ly;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // a wave is one tile row: wall rows, and the rows of an overhanging last
  // tile row (OVER, periodic y only) that lie beyond n_y, are wave-uniform
  const bool live = !OVER || y0 + wave < k.n1;
  const bool wall_lo = WALLY && k.w1 && y0 == 0, wall_hi = WALLY && k.w1 && y0 + TY == k.n1;
  // +1: the populations with c_y = +1 arrive through the wall below, -1: those
  // with c_y = -1 through the wall above, 0: no wall next to this row
  const int wall_side = (wall_lo && wave == 0) ? 1 : ((wall_hi && wave == TY - 1) ? -1 : 0);

  float* anom = reinterpret_cast<float*>(smem + 2 * STAGE);
  auto QX = [&](int b, int slot) -> float& { return anom[b * LXF + slot]; };
  auto QY = [&](int b, int slot) -> float& { return anom[2 * LXF + b * LYF + slot]; };
  // anomaly slots of the node and of its tiled-axis neighbours (periodic, full tiles)
  const int sx_own = ly * (TX + 2) + lx + 1, sxm = sx_own - 1, sxp = sx_own + 1;
  const int sy_own = (ly + 1) * TX + lx, sym = sy_own - TX, syp = sy_own + TX;

  // halo node of this thread: tid < 128 the rows y0 - 1 and y0 + TY, then the
  // columns x0 - 1 and x0 + 64 (tile-local coordinates hx, hy); none beyond a
  // wall
  bool has_halo = tid < 2 * TX + 2 * TY;
  int hx = 0, hy = 0, hslot = 0, hax = 0, h_side = 0;
  if (tid < 2 * TX) {
    const int side = tid >> 6;
    hx = lx;
    hy = side ? TY : -1;
    hslot = (side ? (TY + 1) * TX : 0) + lx;
    hax = 1;
    if (side ? wall_hi : wall_lo) has_halo = false;
  } else if (has_halo) {
    const int q = tid - 2 * TX, side = q / TY, row = q % TY;
    hx = side ? TX : -1;
    hy = row;
    hslot = row * (TX + 2) + (side ? TX + 1 : 0);
    h_side = (wall_lo && row == 0) ? 1 : ((wall_hi && row == TY - 1) ? -1 : 0);
  }
  // in-plane byte offsets of the node and of its halo node (bounce-back
  // loads); a row beyond n_y has an offset past the plane, used only by its
  // stores, which are dropped
  const uint32_t own = uint32_t(gy * k.n0 + gx) * 2u;
  const int hgx = x0 + hx < 0 ? x0 + hx + k.n0 : (x0 + hx >= k.n0 ? x0 + hx - k.n0 : x0 + hx);
  const uint32_t hown = uint32_t((y0 + max(hy, 0)) * k.n0 + hgx) * 2u;
  const float h_uref = hax == 0 ? k.uref[0] : k.uref[1];
  const float h_anom = hax == 0 ? k.anom[0] : k.anom[1];
  const int hofs = hax == 0 ? 0 : 2 * LXF;  // the halo's axis: buffer 0, and the offset to buffer 1
  const int hstep = hax == 0 ? LXF : LYF;

  // LDS read bases (bytes within a stage) per c_x, of the node and of its halo node
  int rb[3], hb[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    rb[c] = col_byte(lx - (c - 1), ly + 1);
    hb[c] = col_byte(hx - (c - 1), hy + 1);
  }
  auto pull_lds = [&](const unsigned char* stg, const int (&base)[3], int i) -> R {
    const int c0 = cq<3>(i, 0);
    return *reinterpret_cast<const R*>(stg + i * BOX + base[c0 + 1]);
  };
  // own post-collision population Q - 1 - i of plane p at in-plane offset off
  auto bounce = [&](int p, uint32_t sb, uint32_t off, int i) -> R {
    return Store<S>::load(rsrc(src + uint64_t(p) * k.slab_bytes), off, (Q - 1 - i) * sb);
  };
  // the values a node pulls from stage stg (plane p); side selects the
  // directions taken by bounce-back (0: none)
  auto values_side = [&](auto side, const unsigned char* stg, const int (&base)[3], int p, uint32_t sb,
                         uint32_t off, R (&v)[Q]) {
    constexpr int SIDE_ = decltype(side)::value;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      v[i] = SIDE_ != 0 && cq<3>(i, 1) == SIDE_ ? bounce(p, sb, off, i) : pull_lds(stg, base, i);
  };
  using Side0 = std::integral_constant<int, 0>;
  using SideLo = std::integral_constant<int, 1>;
  using SideHi = std::integral_constant<int, -1>;
  auto node_values = [&](int side, const unsigned char* stg, const int (&base)[3], int p, uint32_t sb,
                         uint32_t off, R (&v)[Q]) {
    if (WALLY && side == 1) values_side(SideLo(), stg, base, p, sb, off, v);
    else if (WALLY && side == -1) values_side(SideHi(), stg, base, p, sb, off, v);
    else values_side(Side0(), stg, base, p, sb, off, v);
  };
  // deviation moments of pulled values
  auto moments = [&](const R (&v)[Q], float& dr, float (&djo)[3]) {
    float f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Store<S>::to_float(v[i]);
    float r, m[3];
    Puller<3, S, false>::line_moments(f, S == 1 ? k.one : 1.f, r, m);
    dr = r * k.inv_scale;
    djo[0] = k.mfac[0] * m[0];
    djo[1] = k.mfac[1] * m[1];
    djo[2] = k.mfac[2] * m[2];
  };

  // ---- staging: this wave's direct loads (fixed along the march) ----
  // The stage's wave instructions are taken in rounds of NW: in round t, wave
  // w writes piece kind w % PER_BOX (interior instructions, then the side
  // pairs) of box j = (NW / PER_BOX) t + w / PER_BOX, so a wave's kind, and which of
  // its lanes hold a piece, are fixed. dv is this lane's byte offset within a
  // plane slab for box j (direction j's array and the row and column the
  // piece comes from); the source plane p - c_jz enters through the buffer
  // resource.
  static_assert(NW % PER_BOX == 0, "a wave keeps its piece kind from round to round");
  constexpr int BPR = NW / PER_BOX;  // boxes per round
  constexpr int ROUNDS = (27 + BPR - 1) / BPR;
  const int kind = wave % PER_BOX, jw = wave / PER_BOX;
  const bool side_kind = kind == IINSTR;
  const bool dok = side_kind ? lx < SITEMS : 64 * kind + lx < IITEMS;
  uint32_t dv[ROUNDS];
#pragma unroll
  for (int t = 0; t < ROUNDS; ++t) {
    const int j = min(BPR * t + jw, 26);
    const int c1 = cq<3>(j, 1);
    if (!side_kind) {
      const int it = 64 * kind + lx;
      const int r = min(it >> 3, ROWS - 1), q = it & 7;
      dv[t] = uint32_t(j) * sb0 + uint32_t(wrap(y0 - 1 - c1 + r, k.n1) * k.n0 + x0) * 2u + 16u * q;
    } else {
      const int r = min(lx >> 1, ROWS - 1), side = lx & 1;
      const int xs = side ? (x0 + TX == k.n0 ? 0 : x0 + TX) : (x0 == 0 ? k.n0 - 2 : x0 - 2);
      dv[t] = uint32_t(j) * sb0 + uint32_t(wrap(y0 - 1 - c1 + r, k.n1) * k.n0 + xs) * 2u;
    }
  }
  const int kind_off = side_kind ? SIDE : 1024 * kind;
  // issues the direct loads of the stage of node plane p (direction j from
  // plane p - c_jz) into stage stg
  auto stage_load = [&](int p, unsigned char* stg) {
    const char* base[3];  // slab of plane p - c_z, c_z = -1, 0, 1
#pragma unroll
    for (int c = 0; c < 3; ++c) base[c] = src + uint64_t(wrap(p - (c - 1), k.n2)) * k.slab_bytes;
    if (dok) {
#pragma unroll
      for (int t = 0; t < ROUNDS; ++t) {
        const int j = BPR * t + jw;
        if (BPR * (t + 1) <= 27 || j < 27) {
          // the z group of box j: fixed for a round whose boxes share it
          const int g_lo = BPR * t / 9, g_hi = (BPR * t + BPR - 1) / 9;  // constants after unrolling
          const int g = g_lo == g_hi ? g_lo : j / 9;
          const Rsrc rs = rsrc(g == 0 ? base[0] : (g == 1 ? base[1] : base[2]));
          const lds_ptr to = (lds_ptr)stg + j * BOX + kind_off;
          if (side_kind) __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, to, 4, dv[t], 0, 0, 0);
          else __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, to, 16, dv[t], 0, 0, 0);
        }
      }
    }
  };

  // values, moments and anomalies of the node at a staged plane, and the
  // halo node's anomaly into exchange buffer bo
  float drho, dj[3], qc[3] = {0.f, 0.f, 0.f}, qprev;
  Held held;  // values of the plane being relaxed
  auto plane_pass = [&](const unsigned char* stg, int p, uint32_t sb, int bo, float& dr, float (&djo)[3],
                        float (&q)[3], Held& keep) {
    R v[Q];
    node_values(wall_side, stg, rb, p, sb, own, v);
#pragma unroll
    for (int w = 0; w < 14; ++w)
      keep.w[w] = uint32_t(v[2 * w]) | (2 * w + 1 < Q ? uint32_t(v[2 * w + 1]) << 16 : 0u);
    moments(v, dr, djo);
    const float ir = recip(1.f + dr);
    q[0] = anomaly(k, 0, djo[0], ir);
    q[1] = anomaly(k, 1, djo[1], ir);
    q[2] = anomaly(k, 2, djo[2], ir);
    if (has_halo) {
      R hv[Q];
      node_values(h_side, stg, hb, p, sb, hown, hv);
      float hr, hj[3];
      moments(hv, hr, hj);
      const float j = h_uref + (hax == 0 ? hj[0] : hj[1]);
      const float u = j * recip(1.f + hr);
      anom[hofs + bo * hstep + hslot] = j * h_anom - j * u * u;
    }
  };
  auto plane_index = [&](int zz) {
    while (zz >= k.n2) zz -= k.n2;
    return zz < 0 ? zz + k.n2 : zz;
  };

  unsigned char* const st0 = smem;
  unsigned char* const st1 = smem + STAGE;
  // ---- prologue: the ring plane before the first, the first plane, and the
  // loads of the second ----
  stage_load(plane_index(zs - dir), st0);
  stage_load(zs, st1);
  drain_vm();
  __syncthreads();
  {
    R v[Q];
    node_values(wall_side, st0, rb, plane_index(zs - dir), sb0, own, v);
    float dr, djp[3];
    moments(v, dr, djp);
    qprev = anomaly(k, 2, djp[2], recip(1.f + dr));
  }
  plane_pass(st1, zs, sb0, 0, drho, dj, qc, held);
  QX(0, sx_own) = qc[0];
  QY(0, sy_own) = qc[1];
  __syncthreads();  // the ring plane's stage is read
  stage_load(plane_index(zs + dir), st0);
  drain_vm();
  __syncthreads();

  const float hz = dir > 0 ? k.hil[2] : -k.hil[2];  // z difference in march order
  // One plane of the march: the stage of the next plane is `nxt` (complete),
  // `fre` receives the plane after it; `cur` holds this plane's values and
  // `held_next` receives the next plane's.
  auto plane_step = [&](int m, unsigned char* nxt, unsigned char* fre, const Held& cur, Held& held_next) {
    const int z = zs + dir * m;
    const int b = m & 1;
    // the array distance is made opaque per plane (see the kernel above)
    uint32_t sb = sb0;
    asm("" : "+s"(sb) : "s"(z));
    // loads of the plane two on in march order fly while this plane is
    // updated (on the last plane there is none that the tile reads)
    if (m + 2 <= len) stage_load(plane_index(z + 2 * dir), fre);

    if constexpr (DIAG) {
      // the record's moments of plane z, from its held pulled values (here,
      // before the next plane's values are held too)
      // (every lane of a live row holds a node: each field is folded as soon
      // as it is formed)
      if (live)
        diag_node<3>(da, [&](int i) { return Store<S>::to_float(cur.get(i)); }, gx, gy, z,
                     int64_t(gx) + int64_t(k.n0) * (int64_t(gy) + int64_t(k.n1) * z),
                     [&](int j, double v) { diag_fold_one(j, v, wslot); });
    }

    // next plane: values (kept for its relaxation), own anomaly (closes the
    // ring) and the halo's
    float drn, djn[3], qn[3];
    plane_pass(nxt, plane_index(z + dir), sb, b ^ 1, drn, djn, qn, held_next);

    // collision of plane z
    {
      float Gd[3];
      Gd[0] = (QX(b, sxp) - QX(b, sxm)) * k.hil[0];
      // beyond a wall the anomaly is the odd ghost of the wall row
      const float qym = wall_side == 1 ? -qc[1] : QY(b, sym);
      const float qyp = wall_side == -1 ? -qc[1] : QY(b, syp);
      Gd[1] = (qyp - qym) * k.hil[1];
      Gd[2] = (qn[2] - qprev) * hz;
      // a row beyond n_y stores through a resource of no records: the
      // hardware's range check drops every store (its values are the
      // wrapped row's, which the first tile row stores)
      const Rsrc rd = rsrc(dst + uint64_t(z) * k.slab_bytes, live ? -1 : 0);
      collide<3, FORCE, S == 0, false>(k, drho, dj, Gd, [&](int i) { return Store<S>::to_float(cur.get(i)); },
                        [&](int i, float o) { Store<S>::store(rd, own, i * sb, o); });
    }
    QX(b ^ 1, sx_own) = qn[0];
    QY(b ^ 1, sy_own) = qn[1];
    // this wave's direct loads are complete; after the barrier every wave's
    // are, and every read of the stage just used is done
    wait_vm_but_stores();
    __syncthreads();
    drho = drn;
    dj[0] = djn[0];
    dj[1] = djn[1];
    dj[2] = djn[2];
    qprev = qc[2];
    qc[0] = qn[0];
    qc[1] = qn[1];
    qc[2] = qn[2];
  };
  unsigned char* nx = st0;
  unsigned char* fr = st1;
  for (int m = 0; m < len; ++m) {
    Held other;
    plane_step(m, nx, fr, held, other);
    held = other;
    unsigned char* const t = nx;
    nx = fr;
    fr = t;
  }
}

template <int S, bool FORCE, bool WALLY, bool DIAG>
__global__ void __launch_bounds__(lds::NT)
    step_kernel_lds(const TableHeader* __restrict__ hdr, const LatticeDesc* __restrict__ table, int64_t substep,
                    DiagArgs da) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[lds::BYTES];
  const int64_t total = hdr->total_tiles;
  const int count = hdr->count;
  const int gpx = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7;
  const int lb = blockIdx.x >> 3;
  const int64_t per = (total + 7) >> 3;
  const int64_t tb = xcd * per;
  const int64_t te = min(tb + per, total);
  __shared__ double wsum[DIAG ? (lds::NT / 64) * kDiagRows * kDF : 1];
  double* const wslot = wsum + (DIAG ? (threadIdx.x >> 6) * kDiagRows * kDF : 0);
  if constexpr (DIAG) diag_slots_init(wslot);
  int L = 0;
  for (int64_t t = tb + lb; t < te; t += gpx) {
    while (L + 1 < count && table[L + 1].tile_base <= t) ++L;
    const LatticeDesc* d = table + L;
    if (substep < d->nsteps) {
      const int parity = (d->parity0 + int(substep & 1)) & 1;
      const int64_t tl = t - d->tile_base;
      // a last tile row that overhangs a periodic y axis takes the variant
      // whose rows beyond n_y store nothing; every other tile the plain one
      if (!WALLY && d->n[1] % lds::TY != 0 && (tl / d->tiles[0]) % d->tiles[1] == d->tiles[1] - 1)
        step_tile_lds<S, FORCE, WALLY, DIAG, !WALLY>(d, tl, parity, smem, da, wslot);
      else
        step_tile_lds<S, FORCE, WALLY, DIAG, false>(d, tl, parity, smem, da, wslot);
    }
    __syncthreads();
  }
  if constexpr (DIAG) diag_block_store<lds::NT / 64>(wsum, da.partials);
}

template <int D, int S, bool WALL, bool FORCE, bool DIAG, bool MRT3>
__global__ void __launch_bounds__(Threads<D>::value)
    step_kernel(const TableHeader* __restrict__ hdr, const LatticeDesc* __restrict__ table, int64_t substep,
                DiagArgs da) {
  __shared__ __attribute__((aligned(16))) float sq[Geo<D, S>::LDS];
  __shared__ double wsum[DIAG ? (Threads<D>::value / 64) * kDiagRows * kDF : 1];
  const int64_t total = hdr->total_tiles;
  const int count = hdr->count;
  const int gpx = gridDim.x >> 3;  // blocks per XCD (grid is a multiple of 8)
  const int xcd = blockIdx.x & 7;
  const int lb = blockIdx.x >> 3;
  const int64_t per = (total + 7) >> 3;
  const int64_t tb = xcd * per;
  const int64_t te = min(tb + per, total);
  double* const wslot = wsum + (DIAG ? (threadIdx.x >> 6) * kDiagRows * kDF : 0);
  if constexpr (DIAG) diag_slots_init(wslot);
  int L = 0;
  for (int64_t t = tb + lb; t < te; t += gpx) {
    while (L + 1 < count && table[L + 1].tile_base <= t) ++L;
    const LatticeDesc* d = table + L;
    if (substep < d->nsteps) {
      const int parity = (d->parity0 + int(substep & 1)) & 1;
      step_tile<D, S, WALL, FORCE, DIAG, MRT3>(d, t - d->tile_base, parity, sq, da, wslot);
    }
    __syncthreads();
  }
  if constexpr (DIAG) diag_block_store<Threads<D>::value / 64>(wsum, da.partials);
}

template <int D, int S, bool WALL, bool FORCE, bool MRT3>
hipError_t launch_one(const TableHeader* hdr, const LatticeDesc* table, int64_t substep, int grid,
                      const DiagArgs* da, hipStream_t st) {
  if (da)
    hipLaunchKernelGGL((step_kernel<D, S, WALL, FORCE, true, MRT3>), dim3(grid), dim3(Geo<D, S>::NT), 0, st, hdr,
                       table, substep, *da);
  else
    hipLaunchKernelGGL((step_kernel<D, S, WALL, FORCE, false, MRT3>), dim3(grid), dim3(Geo<D, S>::NT), 0, st, hdr,
                       table, substep, DiagArgs{});
  return hipGetLastError();
}

template <int D, int S, bool MRT3>
hipError_t launch_ds(bool wall, bool force, const TableHeader* hdr, const LatticeDesc* table, int64_t s,
                     int grid, const DiagArgs* da, hipStream_t st) {
  if (wall) {
    return force ? launch_one<D, S, true, true, MRT3>(hdr, table, s, grid, da, st)
                 : launch_one<D, S, true, false, MRT3>(hdr, table, s, grid, da, st);
  }
  return force ? launch_one<D, S, false, true, MRT3>(hdr, table, s, grid, da, st)
               : launch_one<D, S, false, false, MRT3>(hdr, table, s, grid, da, st);
}

template <int S, bool FORCE, bool WALLY>
hipError_t launch_lds(const TableHeader* hdr, const LatticeDesc* table, int64_t substep, int grid,
                      const DiagArgs* da, hipStream_t st) {
  if (da)
    hipLaunchKernelGGL((step_kernel_lds<S, FORCE, WALLY, true>), dim3(grid), dim3(lds::NT), 0, st, hdr, table,
                       substep, *da);
  else
    hipLaunchKernelGGL((step_kernel_lds<S, FORCE, WALLY, false>), dim3(grid), dim3(lds::NT), 0, st, hdr, table,
                       substep, DiagArgs{});
  return hipGetLastError();
}

template <int S>
hipError_t launch_lds_s(bool wall, bool force, const TableHeader* hdr, const LatticeDesc* table, int64_t s,
                        int grid, const DiagArgs* da, hipStream_t st) {
  if (wall) return force ? launch_lds<S, true, true>(hdr, table, s, grid, da, st)
                         : launch_lds<S, false, true>(hdr, table, s, grid, da, st);
  return force ? launch_lds<S, true, false>(hdr, table, s, grid, da, st)
               : launch_lds<S, false, false>(hdr, table, s, grid, da, st);
}

}  // namespace

int step_block_threads(int kind) {
  return kind == kKindD3Staged ? lds::NT : (kind == kKindD2 ? Geo<2, 0>::NT : Geo<3, 0>::NT);
}

template <int D, int S, bool WALL, bool FORCE, bool MRT3>
int occupancy_one() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<D, S, WALL, FORCE, false, MRT3>, Geo<D, S>::NT,
                                                   0) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <int S, bool FORCE, bool WALLY>
int occupancy_lds() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel_lds<S, FORCE, WALLY, false>, lds::NT, 0) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <int S>
int occupancy_lds_s(bool wall, bool force) {
  if (wall) return force ? occupancy_lds<S, true, true>() : occupancy_lds<S, false, true>();
  return force ? occupancy_lds<S, true, false>() : occupancy_lds<S, false, false>();
}

template <int D, int S, bool MRT3>
int occupancy_ds(bool wall, bool force) {
  if (wall) return force ? occupancy_one<D, S, true, true, MRT3>() : occupancy_one<D, S, true, false, MRT3>();
  return force ? occupancy_one<D, S, false, true, MRT3>() : occupancy_one<D, S, false, false, MRT3>();
}

template <int D, bool MRT3>
int occupancy_s(int storage, bool wall, bool force) {
  switch (storage) {
    case 0: return occupancy_ds<D, 0, MRT3>(wall, force);
    case 1: return occupancy_ds<D, 1, MRT3>(wall, force);
    default: return occupancy_ds<D, 2, MRT3>(wall, force);
  }
}

int step_blocks_per_cu(int kind, int storage, bool wall, bool force) {
  switch (kind) {
    case kKindD3Staged:
      return storage == 1 ? occupancy_lds_s<1>(wall, force) : occupancy_lds_s<2>(wall, force);
    case kKindD3: return occupancy_s<3, false>(storage, wall, force);
    case kKindD3Mrt: return occupancy_s<3, true>(storage, wall, force);
    default: return occupancy_s<2, false>(storage, wall, force);
  }
}

namespace {
template <int D, bool MRT3>
hipError_t launch_s(int storage, bool wall, bool force, const TableHeader* hdr, const LatticeDesc* table,
                    int64_t substep, int grid, const DiagArgs* da, hipStream_t st) {
  switch (storage) {
    case 0: return launch_ds<D, 0, MRT3>(wall, force, hdr, table, substep, grid, da, st);
    case 1: return launch_ds<D, 1, MRT3>(wall, force, hdr, table, substep, grid, da, st);
    case 2: return launch_ds<D, 2, MRT3>(wall, force, hdr, table, substep, grid, da, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_any(int kind, int storage, bool wall, bool force, const TableHeader* hdr,
                      const LatticeDesc* table, int64_t substep, int grid, const DiagArgs* da, hipStream_t st) {
  if (grid <= 0 || (grid & 7)) return hipErrorInvalidConfiguration;
  switch (kind) {
    case kKindD3Staged:
      // (wall: bounce-back on y only; the host admits no other walls here)
      if (storage != 1 && storage != 2) return hipErrorInvalidValue;
      return storage == 1 ? launch_lds_s<1>(wall, force, hdr, table, substep, grid, da, st)
                          : launch_lds_s<2>(wall, force, hdr, table, substep, grid, da, st);
    case kKindD3: return launch_s<3, false>(storage, wall, force, hdr, table, substep, grid, da, st);
    case kKindD3Mrt: return launch_s<3, true>(storage, wall, force, hdr, table, substep, grid, da, st);
    case kKindD2: return launch_s<2, false>(storage, wall, force, hdr, table, substep, grid, da, st);
  }
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_step(int kind, int storage, bool wall, bool force, const TableHeader* hdr,
                       const LatticeDesc* table, int64_t substep, int grid, hipStream_t st) {
  return launch_any(kind, storage, wall, force, hdr, table, substep, grid, nullptr, st);
}

hipError_t launch_step_diag(int kind, int storage, bool wall, bool force, const TableHeader* hdr,
                            const LatticeDesc* table, int64_t substep, int grid, const DiagArgs& da,
                            hipStream_t st) {
  if (grid > kDiagBlocks || !da.ustage || !da.partials) return hipErrorInvalidValue;
  return launch_any(kind, storage, wall, force, hdr, table, substep, grid, &da, st);
}

}  // namespace elbm
