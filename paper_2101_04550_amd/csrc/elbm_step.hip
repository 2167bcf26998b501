// Fused extended-LBGK step kernel for gfx950.
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
// Populations are Q structure-of-arrays arrays (x fastest), two buffers
// (ping-pong). A block owns a tile of 64 x 8 nodes of the x-y plane (D3Q27)
// or a 256-node x strip (D2Q9) and marches along the slowest axis (z, resp.
// y) over `chunk` planes. The anomaly of the marched axis comes from a
// three-plane register ring (previous, current, next); the anomalies of the
// tiled axes go through LDS, double buffered by plane, with a one-node cross
// halo whose nodes are pulled by the first threads of the block. Each plane
// costs one HBM read and one HBM write of every population of its nodes;
// halo and ring-end pulls re-read data neighbouring tiles also read (L2).
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

#include "elbm_internal.h"

namespace elbm {
namespace {

// Storage formats through their raw bits: FP32 values, or the 16 bits of an
// FP16 / BF16 value (deviations scaled by the lattice's storage scale).
// Stores bypass cache allocation: a step's output is not read again until the
// next launch.
template <int S>
struct Store;

template <>
struct Store<0> {
  using T = float;
  using R = float;
  __device__ static __forceinline__ R load_raw(const T* p) { return *p; }
  __device__ static __forceinline__ float to_float(R r) { return r; }
  __device__ static __forceinline__ void store(T* p, float v) { __builtin_nontemporal_store(v, p); }
};

template <>
struct Store<1> {
  using T = __half;
  using R = unsigned short;
  __device__ static __forceinline__ R load_raw(const T* p) { return *reinterpret_cast<const R*>(p); }
  __device__ static __forceinline__ float to_float(R r) { return __half2float(__ushort_as_half(r)); }
  __device__ static __forceinline__ void store(T* p, float v) {
    __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v)), reinterpret_cast<R*>(p));
  }
};

template <>
struct Store<2> {
  using T = __hip_bfloat16;
  using R = unsigned short;
  __device__ static __forceinline__ R load_raw(const T* p) { return *reinterpret_cast<const R*>(p); }
  __device__ static __forceinline__ float to_float(R r) { return __uint_as_float(unsigned(r) << 16); }
  __device__ static __forceinline__ void store(T* p, float v) {
    __builtin_nontemporal_store(__bfloat16_as_ushort(__float2bfloat16(v)), reinterpret_cast<R*>(p));
  }
};

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
  int n0, n1, n2, plane;
  int64_t stride;
  bool w0, w1, w2;
  float lam[3], inv_lam[3], inv_lam2[3], hil[3], mfac[3], anom[3], uref[3], g[3];
  float W[3][3], WW[3][3];
  float omega, coef, inv_scale, scale, om1, oms;
};

// Pulled populations of one node in storage format (FP32 value, or the raw
// 16 bits of an FP16 / BF16 value).
template <int S, int Q>
struct Pops {
  typename Store<S>::R v[Q];
  __device__ __forceinline__ float get(int i) const { return Store<S>::to_float(v[i]); }
};

template <int D, int S, bool WALL>
struct Puller {
  using T = typename Store<S>::T;
  static constexpr int Q = Geo<D, S>::Q;

  // Pulls the populations arriving at node (x, y, z) (all in range) and forms
  // the deviation moments drho = sum h, dj_a = lambda_a sum c_ia h. With KEEP
  // the pulled values are kept (in storage format) in h.
  template <bool KEEP>
  __device__ static __forceinline__ void pull(const TileConst& k, const T* __restrict__ src, int x,
                                              int y, int z, Pops<S, Q>& h, float& drho, float (&dj)[3]) {
    int sx[3], sy[3], sz[3];
    bool ox[3], oy[3], oz[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int ax = x - (c - 1), ay = y - (c - 1), az = z - (c - 1);
      ox[c] = WALL && k.w0 && (ax < 0 || ax >= k.n0);
      oy[c] = WALL && k.w1 && (ay < 0 || ay >= k.n1);
      oz[c] = WALL && k.w2 && (az < 0 || az >= k.n2);
      sx[c] = wrap(ax, k.n0);
      sy[c] = (D == 3) ? wrap(ay, k.n1) * k.n0 : 0;
      sz[c] = wrap(az, k.n2) * k.plane;
    }
    const int own = x + k.n0 * (y + k.n1 * z);
    float v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int c0 = cq<D>(i, 0), c1 = cq<D>(i, 1), c2 = cq<D>(i, 2);
      const int o = sx[c0 + 1] + sy[c1 + 1] + sz[c2 + 1];
      auto raw = Store<S>::load_raw(src + i * k.stride + o);
      if (WALL) {
        const bool out = (c0 != 0 && ox[c0 + 1]) || (c1 != 0 && oy[c1 + 1]) || (c2 != 0 && oz[c2 + 1]);
        if (out) raw = Store<S>::load_raw(src + (Q - 1 - i) * k.stride + own);
      }
      if (KEEP) h.v[i] = raw;
      v[i] = Store<S>::to_float(raw);
    }
    float r, m[3];
    line_moments(v, r, m);
    // values are in storage scale: the factors carry 1/scale
    drho = r * k.inv_scale;
    dj[0] = k.mfac[0] * m[0];
    dj[1] = k.mfac[1] * m[1];
    dj[2] = k.mfac[2] * m[2];
  }

  // Moments of the 3^D values in lattice order: sums along x-lines of three
  // first, then combined (fewer additions than direction by direction).
  __device__ static __forceinline__ void line_moments(const float (&v)[Q], float& r, float (&m)[3]) {
    if (D == 3) {
      float s[3][3], jx = 0.f;
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2)
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) {
          const int b = 3 * k1 + 9 * k2;
          s[k1][k2] = (v[b] + v[b + 1]) + v[b + 2];
          jx += v[b + 2] - v[b];
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
        s[k2] = (v[b] + v[b + 1]) + v[b + 2];
        jx += v[b + 2] - v[b];
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

template <int D, int S, bool WALL, bool FORCE>
__device__ __forceinline__ void step_tile(const LatticeDesc* __restrict__ Ld, int64_t tl, int parity,
                                          float* __restrict__ sq) {
  using G = Geo<D, S>;
  using T = typename Store<S>::T;
  using P = Puller<D, S, WALL>;
  constexpr int Q = G::Q, TXW = G::TXW, TYR = G::TYR;

  TileConst k;
  k.n0 = Ld->n[0];
  k.n1 = Ld->n[1];
  k.n2 = Ld->n[2];
  k.plane = k.n0 * k.n1;
  k.stride = Ld->stride;
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
  const T* __restrict__ src = static_cast<const T*>(Ld->buf[parity]);
  T* __restrict__ dst = static_cast<T*>(Ld->buf[parity ^ 1]);

  const int tiles0 = Ld->tiles[0], tiles1 = Ld->tiles[1], chunk = Ld->chunk;
  const int t0 = int(tl % tiles0);
  const int64_t rr = tl / tiles0;
  const int t1 = int(rr % tiles1);
  const int t2 = int(rr / tiles1);
  const int x0 = t0 * TXW, y0 = t1 * TYR;
  const int z0 = t2 * chunk;
  const int z1 = min(z0 + chunk, k.n2);
  const int xe = min(x0 + TXW, k.n0), ye = min(y0 + TYR, k.n1);

  const int tid = threadIdx.x;
  const int lx = D == 3 ? (tid & 63) : tid;
  const int ly = D == 3 ? (tid >> 6) : 0;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool active = gx < k.n0 && gy < k.n1;

  float* qxb[2] = {sq, sq + G::LX};
  float* qyb[2] = {sq + 2 * G::LX, sq + 2 * G::LX + G::LY};

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
  float* hbase = hax == 0 ? sq : sq + 2 * G::LX;  // buffer 0 of the halo's axis
  const int hstep = hax == 0 ? G::LX : G::LY;     // offset to buffer 1

  // the halo node's axis is a run-time value: select its constants once
  const float h_uref = hax == 0 ? k.uref[0] : k.uref[1];
  const float h_anom = hax == 0 ? k.anom[0] : k.anom[1];
  auto halo = [&](int z, int b) {
    if (has_halo) {
      float dr, dj[3];
      Pops<S, Q> unused;
      P::template pull<false>(k, src, hx, hy, z, unused, dr, dj);
      const float ir = recip(1.f + dr);
      const float j = h_uref + (hax == 0 ? dj[0] : dj[1]);
      const float u = j * ir;
      hbase[b * hstep + hslot] = j * h_anom - j * u * u;
    }
  };

  const int cx = active ? gx : 0, cy = active ? gy : 0;

  // ---- prologue: plane before the chunk (ring) and the first plane ----
  Pops<S, Q> h, hn;
  float drho = 0.f, dj[3] = {0.f, 0.f, 0.f};
  float qc[3] = {0.f, 0.f, 0.f};  // anomaly of the current plane at this node
  float qprev = 0.f;
  bool ghost_prev = false;
  {
    int zp = z0 - 1;
    if (z0 == 0) { if (k.w2) ghost_prev = true; else zp = k.n2 - 1; }
    if (active && !ghost_prev) {
      float dr, djp[3];
      P::template pull<false>(k, src, cx, cy, zp, hn, dr, djp);
      qprev = anomaly(k, 2, djp[2], recip(1.f + dr));
    }
    if (active) {
      P::template pull<true>(k, src, cx, cy, z0, h, drho, dj);
      const float ir = recip(1.f + drho);
      qc[0] = anomaly(k, 0, dj[0], ir);
      if (D == 3) qc[1] = anomaly(k, 1, dj[1], ir);
      qc[2] = anomaly(k, 2, dj[2], ir);
      if (ghost_prev) qprev = -qc[2];
      qxb[0][sx_own] = qc[0];
      if (D == 3) qyb[0][sy_own] = qc[1];
    }
    halo(z0, 0);
  }
  __syncthreads();

  for (int z = z0; z < z1; ++z) {
    const int b = (z - z0) & 1;
    // next plane (always pulled: its anomaly closes the ring)
    int zn = z + 1;
    bool ghost_next = false;
    if (zn >= k.n2) { if (k.w2) ghost_next = true; else zn = 0; }
    float drn = 0.f, djn[3] = {0.f, 0.f, 0.f}, qn[3] = {0.f, 0.f, 0.f};
    const bool more = z + 1 < z1;
    if (active && !ghost_next) {
      P::template pull<true>(k, src, cx, cy, zn, hn, drn, djn);
      const float ir = recip(1.f + drn);
      qn[0] = anomaly(k, 0, djn[0], ir);
      if (D == 3) qn[1] = anomaly(k, 1, djn[1], ir);
      qn[2] = anomaly(k, 2, djn[2], ir);
    }
    if (more) halo(z + 1, b ^ 1);
    const float qnext = ghost_next ? -qc[2] : qn[2];

    if (active) {
      // ---- collision of plane z ----
      const float* qx = qxb[b];
      const float qxm = gxm ? -qc[0] : qx[sxm];
      const float qxp = gxp ? -qc[0] : qx[sxp];
      float Gd[3];
      Gd[0] = (qxp - qxm) * k.hil[0];
      Gd[1] = 0.f;
      if (D == 3) {
        const float* qy = qyb[b];
        const float qym = gym ? -qc[1] : qy[sym];
        const float qyp = gyp ? -qc[1] : qy[syp];
        Gd[1] = (qyp - qym) * k.hil[1];
      }
      Gd[2] = (qnext - qprev) * k.hil[2];

      const float rho = 1.f + drho;
      const float ir = recip(rho);
      float du[3], dP[3], d[3][3], p[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (D == 2 && a == 1) {
          du[a] = 0.f;
          dP[a] = 0.f;
        } else {
          du[a] = (dj[a] - drho * k.uref[a]) * ir;
          const float u = k.uref[a] + du[a];
          dP[a] = du[a] * (u + k.uref[a]) + k.coef * Gd[a] * ir;
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

      const int own = cx + k.n0 * (cy + k.n1 * z);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int c0 = cq<D>(i, 0) + 1, c1 = cq<D>(i, 1) + 1, c2 = cq<D>(i, 2) + 1;
        float hs, fr = 0.f;
        if (D == 3) {
          const float X = p[0][c0] * p[1][c1];
          const float dX = d[0][c0] * p[1][c1] + k.W[0][c0] * d[1][c1];
          const float B = X * p[2][c2];
          const float dB = dX * p[2][c2] + k.WW[c0][c1] * d[2][c2];
          hs = drho * B + dB;
          if (FORCE) {
            const float Y = pe[0][c0] * pe[1][c1];
            const float dY = e[0][c0] * (pe[1][c1] + e[1][c1]) + pe[0][c0] * e[1][c1];
            fr = rho * (dY * (pe[2][c2] + e[2][c2]) + Y * e[2][c2]);
          }
        } else {
          const float X = p[0][c0] * p[2][c2];
          const float dX = d[0][c0] * p[2][c2] + k.W[0][c0] * d[2][c2];
          hs = drho * X + dX;
          if (FORCE) fr = rho * (e[0][c0] * (pe[2][c2] + e[2][c2]) + pe[0][c0] * e[2][c2]);
        }
        // relaxation (Sec. 2.1, eq. LBGK) in storage scale:
        // o = (1 - w) h + w scale f* (+ scale F)
        float o = k.om1 * h.get(i) + k.oms * hs;
        if (FORCE) o += k.scale * fr;
        Store<S>::store(dst + i * k.stride + own, o);
      }
    }

    if (more && active) {
      qxb[b ^ 1][sx_own] = qn[0];
      if (D == 3) qyb[b ^ 1][sy_own] = qn[1];
    }
    __syncthreads();
    h = hn;
    drho = drn;
    dj[0] = djn[0];
    dj[1] = djn[1];
    dj[2] = djn[2];
    qprev = qc[2];
    qc[0] = qn[0];
    qc[1] = qn[1];
    qc[2] = qnext;
  }
}

template <int D, int S, bool WALL, bool FORCE>
__global__ void __launch_bounds__(Threads<D>::value)
    step_kernel(const TableHeader* __restrict__ hdr, const LatticeDesc* __restrict__ table, int64_t substep) {
  __shared__ float sq[Geo<D, S>::LDS];
  const int64_t total = hdr->total_tiles;
  const int count = hdr->count;
  const int gpx = gridDim.x >> 3;  // blocks per XCD (grid is a multiple of 8)
  const int xcd = blockIdx.x & 7;
  const int lb = blockIdx.x >> 3;
  const int64_t per = (total + 7) >> 3;
  const int64_t tb = xcd * per;
  const int64_t te = min(tb + per, total);
  int L = 0;
  for (int64_t t = tb + lb; t < te; t += gpx) {
    while (L + 1 < count && table[L + 1].tile_base <= t) ++L;
    const LatticeDesc* d = table + L;
    if (substep < d->nsteps) {
      const int parity = (d->parity0 + int(substep & 1)) & 1;
      step_tile<D, S, WALL, FORCE>(d, t - d->tile_base, parity, sq);
    }
    __syncthreads();
  }
}

template <int D, int S, bool WALL, bool FORCE>
hipError_t launch_one(const TableHeader* hdr, const LatticeDesc* table, int64_t substep, int grid,
                      hipStream_t st) {
  hipLaunchKernelGGL((step_kernel<D, S, WALL, FORCE>), dim3(grid), dim3(Geo<D, S>::NT), 0, st, hdr, table,
                     substep);
  return hipGetLastError();
}

template <int D, int S>
hipError_t launch_ds(bool wall, bool force, const TableHeader* hdr, const LatticeDesc* table, int64_t s,
                     int grid, hipStream_t st) {
  if (wall) {
    return force ? launch_one<D, S, true, true>(hdr, table, s, grid, st)
                 : launch_one<D, S, true, false>(hdr, table, s, grid, st);
  }
  return force ? launch_one<D, S, false, true>(hdr, table, s, grid, st)
               : launch_one<D, S, false, false>(hdr, table, s, grid, st);
}

}  // namespace

int step_block_threads(int D) { return D == 3 ? Geo<3, 0>::NT : Geo<2, 0>::NT; }

template <int D, int S, bool WALL, bool FORCE>
int occupancy_one() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<D, S, WALL, FORCE>, Geo<D, S>::NT, 0) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <int D, int S>
int occupancy_ds(bool wall, bool force) {
  if (wall) return force ? occupancy_one<D, S, true, true>() : occupancy_one<D, S, true, false>();
  return force ? occupancy_one<D, S, false, true>() : occupancy_one<D, S, false, false>();
}

int step_blocks_per_cu(int D, int storage, bool wall, bool force) {
  if (D == 3) {
    switch (storage) {
      case 0: return occupancy_ds<3, 0>(wall, force);
      case 1: return occupancy_ds<3, 1>(wall, force);
      default: return occupancy_ds<3, 2>(wall, force);
    }
  }
  switch (storage) {
    case 0: return occupancy_ds<2, 0>(wall, force);
    case 1: return occupancy_ds<2, 1>(wall, force);
    default: return occupancy_ds<2, 2>(wall, force);
  }
}

hipError_t launch_step(int D, int storage, bool wall, bool force, const TableHeader* hdr,
                       const LatticeDesc* table, int64_t substep, int grid, hipStream_t st) {
  if (grid <= 0 || (grid & 7)) return hipErrorInvalidConfiguration;
  if (D == 3) {
    switch (storage) {
      case 0: return launch_ds<3, 0>(wall, force, hdr, table, substep, grid, st);
      case 1: return launch_ds<3, 1>(wall, force, hdr, table, substep, grid, st);
      case 2: return launch_ds<3, 2>(wall, force, hdr, table, substep, grid, st);
    }
  } else if (D == 2) {
    switch (storage) {
      case 0: return launch_ds<2, 0>(wall, force, hdr, table, substep, grid, st);
      case 1: return launch_ds<2, 1>(wall, force, hdr, table, substep, grid, st);
      case 2: return launch_ds<2, 2>(wall, force, hdr, table, substep, grid, st);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace elbm
