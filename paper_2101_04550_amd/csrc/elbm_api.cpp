// C ABI of the extended-LBGK library: parameter checks, device memory layout,
// handles, the step loop, field/population transfer, diagnostics,
// checkpoints and the batched multi-lattice runner. See include/elbm.h.
#include "elbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "elbm_internal.h"

using namespace elbm;

struct elbm_lattice {
  elbm_params p;
  int D = 0, Q = 0, device = 0;
  int64_t N = 0, pstride = 0, plane = 0, nplanes = 0;
  size_t es = 4, pop_bytes = 0;
  char* base = nullptr;
  void* buf[2] = {nullptr, nullptr};
  TableHeader* hdr_dev = nullptr;
  LatticeDesc* desc_dev = nullptr;
  double* partials = nullptr;  // 2 kDiagBlocks records: moment sums, then enstrophy sums
  float* ustage = nullptr;     // 3 N floats (diag_every > 0): velocity staged by the sample steps
  double* mode_tab = nullptr;  // per-axis mode factors (diag_every > 0)
  double* history = nullptr;
  double* last = nullptr;
  int64_t* hist_count = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;
  int64_t step = 0;
  int64_t ntiles = 0;
  bool wall = false, force = false, staged = false;
  int kind = kKindD2;  // step kernel family (StepKind)
  LatticeDesc desc{};
  LatticeConst64 c64{};
  DiagArgs dargs{};
};

struct elbm_batch_s {
  int capacity = 0, device = 0;
  hipStream_t caller = nullptr;  // ordering only: the batch waits for it and it waits for the batch
  hipStream_t stream = nullptr;  // the batch's own non-blocking stream (capturable)
  hipEvent_t entry = nullptr;
  hipEvent_t copied = nullptr;
  hipEvent_t done = nullptr;
  bool copy_pending = false;
  // one table per kernel class: header followed by `capacity` descriptors
  std::map<int, char*> dev_tables;
  char* host_stage = nullptr;  // pinned, kClasses tables
  std::map<std::tuple<uint64_t, int64_t, std::vector<int>>, hipGraphExec_t> graphs;
};

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string& msg) {
  g_err = msg;
  return code;
}

int32_t hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return ELBM_EDEVICE;
}

#define HIPCHK(call)                                     \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #call);    \
  } while (0)

constexpr int kClasses = kKinds * 12;  // kernel kind (4) x storage (3) x wall (2) x force (2)
constexpr size_t kAlign = 256;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int class_of(int kind, int storage, bool wall, bool force) {
  return ((kind * 3 + storage) * 2 + (wall ? 1 : 0)) * 2 + (force ? 1 : 0);
}
static_assert(kClasses == kStaticClasses, "one static table per kernel class");

// The kernel class of index c (inverse of class_of).
struct ClassKey {
  int kind, storage;
  bool wall, force;
};
ClassKey class_key(int c) { return ClassKey{c / 12, (c / 4) % 3, (c / 2) % 2 == 1, c % 2 == 1}; }

// Persistent grid of a batched launch: a power of two >= the tiles (capped),
// so that one captured graph serves every mix of the same size class.
int batch_grid(int64_t tiles) {
  int64_t g = 64;
  while (g < tiles && g < 4096) g *= 2;
  return int(g);
}

// Whether a lattice takes the LDS-staged step kernel: D3Q27 LBGK with 16-bit
// storage, n_x % 64 == 0, x and z periodic, y bounce-back with
// n_y % kRowsStaged == 0 or periodic with n_y > kRowsStaged / 2 (the last tile
// row may overhang the axis; every row it stages lies within one period).
// ELBM_STAGED=0 forces the register-pull kernel (for measurements).
bool use_staged(const elbm_params& p) {
  if (const char* s = std::getenv("ELBM_STAGED"))
    if (s[0] == '0') return false;
  return p.lattice == 27 && p.collision == ELBM_COLLISION_BGK && p.storage != ELBM_STORE_F32 &&
         p.bc[0] == ELBM_BC_PERIODIC &&
         p.bc[2] == ELBM_BC_PERIODIC && p.n[0] % 64 == 0 &&
         (p.bc[1] == ELBM_BC_PERIODIC ? p.n[1] > kRowsStaged / 2 : p.n[1] % kRowsStaged == 0);
}

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Triplet Psi_c(u, P, lambda) (Sec. 2.2, eqs. phi0S, phiPlusS, phiMinusS).
double psi(int c, double u, double P, double lam) {
  if (c == 0) return 1.0 - P / (lam * lam);
  return 0.5 * (c * u / lam + P / (lam * lam));
}

struct Layout {
  int D = 0, Q = 0;
  int64_t N = 0, pstride = 0, plane = 0, nplanes = 0;
  size_t es = 4, pop_bytes = 0;
  size_t off_buf[2] = {0, 0};
  size_t off_hdr = 0, off_desc = 0, off_partials = 0, off_ustage = 0, off_modetab = 0, off_hist = 0, off_last = 0,
         off_count = 0, total = 0;
  int64_t modetab_len = 0;  // (cos, sin) pairs: n_x + n_y (+ n_z)
  int32_t capacity = 0;
};

int32_t check(const elbm_params* p) {
  if (!p) return fail(ELBM_EINVAL, "params is NULL");
  if (p->abi_version != ELBM_ABI_VERSION)
    return fail(ELBM_EINVAL, "abi_version " + std::to_string(p->abi_version) + " != " +
                                 std::to_string(ELBM_ABI_VERSION));
  if (p->lattice != 9 && p->lattice != 27) return fail(ELBM_EINVAL, "lattice must be 9 (D2Q9) or 27 (D3Q27)");
  const int D = p->lattice == 27 ? 3 : 2;
  if (D == 2 && p->n[2] != 1) return fail(ELBM_EINVAL, "D2Q9 requires n[2] == 1");
  int64_t N = 1;
  for (int a = 0; a < D; ++a) {
    if (p->n[a] < 1) return fail(ELBM_EINVAL, "extents must be positive");
    if (p->bc[a] != ELBM_BC_PERIODIC && p->bc[a] != ELBM_BC_BOUNCEBACK)
      return fail(ELBM_EINVAL, "bc must be ELBM_BC_PERIODIC or ELBM_BC_BOUNCEBACK");
    if (p->bc[a] == ELBM_BC_PERIODIC && p->n[a] < 3)
      return fail(ELBM_EINVAL, "a periodic axis needs at least 3 nodes");
    if (p->bc[a] == ELBM_BC_BOUNCEBACK && p->n[a] < 2)
      return fail(ELBM_EINVAL, "a bounce-back axis needs at least 2 nodes");
    if (!(p->lambda[a] > 0.0) || !std::isfinite(p->lambda[a]))
      return fail(ELBM_EINVAL, "lambda must be positive and finite");
    if (p->n[a] > (int64_t(1) << 30)) return fail(ELBM_EINVAL, "extent too large");
    N *= p->n[a];
    if (N > std::numeric_limits<int32_t>::max())
      return fail(ELBM_EINVAL, "too many nodes: at most 2^31 - 1 per lattice");
  }
  {
    // one plane slab of the marched axis (Q padded direction arrays) must be
    // addressable with 32-bit byte offsets
    const int64_t plane = D == 3 ? p->n[0] * p->n[1] : p->n[0];
    const int64_t es = p->storage == ELBM_STORE_F32 ? 4 : 2;
    if ((plane + 64) * p->lattice * es >= (int64_t(1) << 32))
      return fail(ELBM_EINVAL, "too many nodes per plane: Q * n_x * n_y (D3Q27) or Q * n_x (D2Q9) times the element "
                               "size must stay below 2^32 bytes");
  }
  if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail(ELBM_EINVAL, "T must be positive and finite");
  if (!(p->omega > 0.0 && p->omega < 2.0)) return fail(ELBM_EINVAL, "omega must lie in (0, 2)");
  for (int a = 0; a < D; ++a) {
    if (!(1.0 - p->T / (p->lambda[a] * p->lambda[a]) > 0.0))
      return fail(ELBM_EINVAL, "rest weight 1 - T/lambda^2 must be positive on every axis (T < lambda_min^2)");
  }
  if (!finite3(p->u_adv) || !finite3(p->force) || !finite3(p->mode_k) || !finite3(p->mode_dir))
    return fail(ELBM_EINVAL, "u_adv, force, mode_k, mode_dir must be finite");
  {
    // A bounced population is the node's own post-collision population of
    // the opposite direction; stored as a deviation from the reference
    // equilibrium w(u_adv), it would need the correction w_opp - w_i, which
    // is nonzero whenever u_adv is. The kernels do not apply it, so walls
    // require the rest state as reference.
    bool wall = false, adv = false;
    for (int a = 0; a < D; ++a) {
      wall = wall || p->bc[a] == ELBM_BC_BOUNCEBACK;
      adv = adv || p->u_adv[a] != 0.0;
    }
    if (wall && adv)
      return fail(ELBM_EUNSUPPORTED, "bounce-back walls require u_adv == 0 (the deviation reference of a walled "
                                     "lattice is the rest equilibrium)");
  }
  if (p->storage < ELBM_STORE_F32 || p->storage > ELBM_STORE_BF16)
    return fail(ELBM_EINVAL, "storage must be ELBM_STORE_F32, ELBM_STORE_F16 or ELBM_STORE_BF16");
  if (p->extended != 0 && p->extended != 1) return fail(ELBM_EINVAL, "extended must be 0 or 1");
  if (p->collision != ELBM_COLLISION_BGK && p->collision != ELBM_COLLISION_MRT)
    return fail(ELBM_EINVAL, "collision must be ELBM_COLLISION_BGK or ELBM_COLLISION_MRT");
  if (p->collision == ELBM_COLLISION_MRT) {
    if (!(p->omega_bulk > 0.0 && p->omega_bulk < 2.0) || !(p->omega_ghost > 0.0 && p->omega_ghost < 2.0))
      return fail(ELBM_EINVAL, "omega_bulk and omega_ghost must lie in (0, 2)");
  }
  if (p->diag_every < 0) return fail(ELBM_EINVAL, "diag_every must be >= 0");
  if (p->diag_every > 0 && (p->diag_capacity < 1 || p->diag_capacity > (1 << 24)))
    return fail(ELBM_EINVAL, "diag_capacity must lie in [1, 2^24] when diag_every > 0");
  return ELBM_OK;
}

Layout layout_of(const elbm_params* p) {
  Layout L;
  L.D = p->lattice == 27 ? 3 : 2;
  L.Q = p->lattice;
  L.N = p->n[0] * p->n[1] * p->n[2];
  L.es = p->storage == ELBM_STORE_F32 ? 4 : 2;
  L.plane = L.D == 3 ? int64_t(p->n[0]) * p->n[1] : p->n[0];
  L.nplanes = L.D == 3 ? p->n[2] : p->n[1];
  L.pstride = int64_t(align_up(size_t(L.plane), 64));
  // (a small tail keeps vector loads near the end of the last slab in range)
  L.pop_bytes = align_up(size_t(L.nplanes) * size_t(L.Q) * size_t(L.pstride) * L.es + 1024, 4096);
  L.capacity = p->diag_every > 0 ? p->diag_capacity : 0;
  size_t o = 0;
  L.off_buf[0] = o;
  o += L.pop_bytes;
  L.off_buf[1] = o;
  o += L.pop_bytes;
  L.off_hdr = o;
  o = align_up(o + sizeof(TableHeader), kAlign);
  L.off_desc = o;
  o = align_up(o + sizeof(LatticeDesc), kAlign);
  L.off_partials = o;
  o = align_up(o + 2 * size_t(kDiagBlocks) * kRec * sizeof(double), kAlign);
  if (p->diag_every > 0) {
    L.off_ustage = o;
    o = align_up(o + 3 * size_t(L.N) * sizeof(float), kAlign);
    for (int a = 0; a < L.D; ++a) L.modetab_len += p->n[a];
    L.off_modetab = o;
    o = align_up(o + 2 * size_t(L.modetab_len) * sizeof(double), kAlign);
  }
  L.off_hist = o;
  o = align_up(o + size_t(L.capacity) * kRec * sizeof(double), kAlign);
  L.off_last = o;
  o = align_up(o + kRec * sizeof(double), kAlign);
  L.off_count = o;
  o = align_up(o + sizeof(int64_t), kAlign);
  L.total = o;
  return L;
}

// Marched-axis chunk. A tile of `chunk` planes costs about chunk + 2 plane
// updates (the ring pulls one plane before and one after the chunk); tiles
// run in rounds of `slots` resident blocks. Pick the number of chunks that
// minimises rounds * (chunk + 2). ELBM_CHUNK overrides (for measurements).
int choose_chunk(int D, int64_t t01, int n2, int64_t slots) {
  if (const char* s = std::getenv("ELBM_CHUNK")) {
    const int v = std::atoi(s);
    if (v > 0) return std::min(v, n2);
  }
  const int minc = std::min(n2, D == 3 ? 16 : 4);
  int best = n2;
  double best_cost = 1e300;
  for (int chunk = n2; chunk >= minc; --chunk) {
    const int64_t nc = (n2 + chunk - 1) / chunk;
    if (chunk != (n2 + nc - 1) / nc) continue;  // only the smallest chunk for each chunk count
    const int64_t rounds = (t01 * nc + slots - 1) / slots;
    const double cost = double(rounds) * double(chunk + 2);
    if (cost < best_cost) {
      best_cost = cost;
      best = chunk;
    }
  }
  return best;
}

void fill_desc(elbm_lattice* h) {
  const elbm_params& p = h->p;
  const int D = h->D;
  LatticeDesc d{};
  // internal axis -> physical axis (-1: absent)
  const int phys[3] = {0, D == 3 ? 1 : -1, D == 3 ? 2 : 1};
  for (int a = 0; a < 3; ++a) {
    const int pa = phys[a];
    const double lam = pa >= 0 ? p.lambda[pa] : 1.0;
    const double ur = pa >= 0 ? p.u_adv[pa] : 0.0;
    d.n[a] = pa >= 0 ? int32_t(p.n[pa]) : 1;
    d.wall[a] = pa >= 0 ? (p.bc[pa] == ELBM_BC_BOUNCEBACK) : 0;
    const double scale = p.storage == ELBM_STORE_F16 ? double(kF16Scale) : 1.0;
    d.lam[a] = float(lam);
    d.inv_lam[a] = float(1.0 / lam);
    d.inv_lam2[a] = float(1.0 / (lam * lam));
    d.half_inv_lam[a] = float(0.5 / lam);
    d.mfac[a] = float(lam / scale);
    d.anom[a] = pa >= 0 ? float(lam * lam - 3.0 * p.T) : 0.f;
    d.uref[a] = float(ur);
    d.g[a] = pa >= 0 ? float(p.force[pa]) : 0.f;
    // reference triplet (Sec. 2.2) at rho = 1, u = uref, P = T + uref^2
    for (int c = -1; c <= 1; ++c)
      d.W[a][c + 1] = pa >= 0 ? float(psi(c, ur, p.T + ur * ur, lam)) : (c == 0 ? 1.f : 0.f);
  }
  for (int c0 = -1; c0 <= 1; ++c0)
    for (int c1 = -1; c1 <= 1; ++c1) {
      const double w0 = psi(c0, p.u_adv[0], p.T + p.u_adv[0] * p.u_adv[0], p.lambda[0]);
      const double w1 = D == 3 ? psi(c1, p.u_adv[1], p.T + p.u_adv[1] * p.u_adv[1], p.lambda[1]) : (c1 == 0);
      d.WW[c0 + 1][c1 + 1] = float(w0 * w1);
    }
  d.T = float(p.T);
  d.omega = float(p.omega);
  d.coef = p.extended ? float((2.0 - p.omega) / (2.0 * p.omega)) : 0.f;
  const double scale = p.storage == ELBM_STORE_F16 ? double(kF16Scale) : 1.0;
  d.om1 = float(1.0 - p.omega);
  d.oms = float(p.omega * scale);
  d.one = 1.f;
  d.mrt = p.collision == ELBM_COLLISION_MRT ? 1 : 0;
  if (d.mrt) {
    d.om1g = float(1.0 - p.omega_ghost);
    d.cdev = float(p.omega_ghost - p.omega);
    d.ciso = float(p.omega_ghost - p.omega_bulk);
    d.coefb = p.extended ? float((2.0 - p.omega_bulk) / (2.0 * p.omega_bulk)) : 0.f;
  }
  d.scale = float(scale);
  d.inv_scale = float(1.0 / scale);
  d.buf[0] = h->buf[0];
  d.buf[1] = h->buf[1];
  d.pstride = h->pstride;
  const int txw = D == 3 ? kTileX3 : 64 * kStrips2;
  const int tyr = D == 3 ? (h->staged ? kRowsStaged : kRows3) : 1;
  d.tiles[0] = (d.n[0] + txw - 1) / txw;
  d.tiles[1] = (d.n[1] + tyr - 1) / tyr;
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus <= 0)
    cus = 256;
  const int bpc = step_blocks_per_cu(h->kind, p.storage, h->wall, h->force);
  d.chunk = choose_chunk(D, int64_t(d.tiles[0]) * d.tiles[1], d.n[2], int64_t(cus) * bpc);
  d.tiles[2] = (d.n[2] + d.chunk - 1) / d.chunk;
  d.ntiles = int64_t(d.tiles[0]) * d.tiles[1] * d.tiles[2];
  d.tile_base = 0;
  d.parity0 = 0;
  d.nsteps = std::numeric_limits<int64_t>::max();
  h->desc = d;
  h->ntiles = d.ntiles;

  LatticeConst64& c = h->c64;
  c = LatticeConst64{};
  c.D = D;
  c.Q = h->Q;
  c.N = h->N;
  c.pstride = h->pstride;
  c.plane = h->plane;
  c.storage = p.storage;
  c.T = p.T;
  c.scale = scale;
  c.inv_scale = 1.0 / scale;
  for (int a = 0; a < 3; ++a) {
    c.n[a] = int32_t(p.n[a]);
    const bool on = a < D;
    c.wall[a] = on ? (p.bc[a] == ELBM_BC_BOUNCEBACK) : 0;
    c.lam[a] = on ? p.lambda[a] : 1.0;
    c.uref[a] = on ? p.u_adv[a] : 0.0;
    c.g[a] = on ? p.force[a] : 0.0;
    c.mode_k[a] = on ? p.mode_k[a] : 0.0;
    c.mode_dir[a] = on ? p.mode_dir[a] : 0.0;
    for (int k = -1; k <= 1; ++k)
      c.W[a][k + 1] = on ? psi(k, c.uref[a], p.T + c.uref[a] * c.uref[a], c.lam[a]) : (k == 0 ? 1.0 : 0.0);
  }
  c.has_mode = (c.mode_dir[0] != 0.0 || c.mode_dir[1] != 0.0 || c.mode_dir[2] != 0.0) ? 1 : 0;
}

void fill_diag_args(elbm_lattice* h) {
  const LatticeConst64& c = h->c64;
  DiagArgs& d = h->dargs;
  d.ustage = h->ustage;
  d.partials = h->partials;
  d.mode_tab = h->mode_tab;
  int32_t off = 0;
  for (int a = 0; a < 3; ++a) {
    d.lam[a] = c.lam[a];
    d.uref[a] = c.uref[a];
    d.g[a] = c.g[a];
    d.mode_dir[a] = c.mode_dir[a];
    d.n[a] = c.n[a];
    d.mode_off[a] = off;
    if (a < h->D) off += c.n[a];
  }
  d.inv_scale = c.inv_scale;
  d.N = c.N;
  d.has_mode = c.has_mode;
}

int grid_for_tiles(int64_t ntiles) {
  const int64_t g = (ntiles + 7) / 8 * 8;
  return int(std::min<int64_t>(std::max<int64_t>(g, 8), int64_t(1) << 30));
}

int32_t set_dev(int dev) {
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != dev) HIPCHK(hipSetDevice(dev));
  return ELBM_OK;
}

void* state_buf(elbm_lattice* h) { return h->buf[h->step & 1]; }
void* spare_buf(elbm_lattice* h) { return h->buf[(h->step & 1) ^ 1]; }

int32_t reset_history(elbm_lattice* h) {
  HIPCHK(hipMemsetAsync(h->hist_count, 0, sizeof(int64_t), h->stream));
  return ELBM_OK;
}

int32_t run_diag(elbm_lattice* h, bool append) {
  HIPCHK(launch_diag(h->c64, state_buf(h), static_cast<float*>(spare_buf(h)), h->partials, h->history,
                     h->hist_count, append ? int32_t(h->p.diag_capacity) : 0, h->last, h->step, h->stream));
  return ELBM_OK;
}

void record_to_diag(const double* r, elbm_diag_record* out) {
  out->step = int64_t(r[R_STEP]);
  out->mass = r[R_MASS];
  out->mom[0] = r[R_MOM0];
  out->mom[1] = r[R_MOM1];
  out->mom[2] = r[R_MOM2];
  out->ke = r[R_KE];
  out->enstrophy = r[R_ENS];
  out->mode_re = r[R_MODE_RE];
  out->mode_im = r[R_MODE_IM];
  out->max_uperp = r[R_MAXU];
  out->min_rho = r[R_MINRHO];
  out->nan_count = int64_t(r[R_NAN]);
}

// Checkpoint: this header, then the raw plane-slab state.
constexpr char kCkptMagic[9] = "ELBMCKP2";

struct CkptHeader {
  char magic[8];
  uint32_t abi;
  uint32_t es;
  int64_t step;
  int64_t pstride;
  int64_t bytes;
  elbm_params params;
};

bool same_problem(const elbm_params& a, const elbm_params& b) {
  return a.lattice == b.lattice && a.n[0] == b.n[0] && a.n[1] == b.n[1] && a.n[2] == b.n[2] &&
         std::memcmp(a.lambda, b.lambda, sizeof a.lambda) == 0 && a.T == b.T && a.omega == b.omega &&
         std::memcmp(a.u_adv, b.u_adv, sizeof a.u_adv) == 0 && std::memcmp(a.force, b.force, sizeof a.force) == 0 &&
         std::memcmp(a.bc, b.bc, sizeof a.bc) == 0 && a.storage == b.storage && a.extended == b.extended &&
         a.collision == b.collision &&
         (a.collision == ELBM_COLLISION_BGK || (a.omega_bulk == b.omega_bulk && a.omega_ghost == b.omega_ghost));
}

}  // namespace

extern "C" {

uint32_t elbm_abi_version(void) { return ELBM_ABI_VERSION; }

const char* elbm_status_string(int32_t s) {
  switch (s) {
    case ELBM_OK: return "ELBM_OK";
    case ELBM_EINVAL: return "ELBM_EINVAL";
    case ELBM_EUNSUPPORTED: return "ELBM_EUNSUPPORTED";
    case ELBM_ENOMEM: return "ELBM_ENOMEM";
    case ELBM_EDEVICE: return "ELBM_EDEVICE";
    case ELBM_EUNSTABLE: return "ELBM_EUNSTABLE";
    default: return "ELBM_UNKNOWN";
  }
}

const char* elbm_last_error(void) { return g_err.c_str(); }

int32_t elbm_validate(const elbm_params* p) { return check(p); }

int32_t elbm_query_bytes(const elbm_params* p, size_t* bytes) {
  if (!bytes) return fail(ELBM_EINVAL, "bytes is NULL");
  const int32_t s = check(p);
  if (s != ELBM_OK) return s;
  *bytes = layout_of(p).total;
  return ELBM_OK;
}

int32_t elbm_create(const elbm_params* p, void* dev_buf, size_t bytes, void* hip_stream, elbm_handle* out) {
  if (!out) return fail(ELBM_EINVAL, "out is NULL");
  *out = nullptr;
  int32_t s = check(p);
  if (s != ELBM_OK) return s;
  const Layout L = layout_of(p);
  if (!dev_buf) return fail(ELBM_EINVAL, "dev_buf is NULL");
  if (reinterpret_cast<uintptr_t>(dev_buf) % kAlign) return fail(ELBM_EINVAL, "dev_buf must be 256-byte aligned");
  if (bytes < L.total)
    return fail(ELBM_ENOMEM, "device buffer holds " + std::to_string(bytes) + " bytes, " + std::to_string(L.total) +
                                 " needed");
  auto* h = new (std::nothrow) elbm_lattice();
  if (!h) return fail(ELBM_EINVAL, "out of host memory");
  h->p = *p;
  h->D = L.D;
  h->Q = L.Q;
  h->N = L.N;
  h->pstride = L.pstride;
  h->plane = L.plane;
  h->nplanes = L.nplanes;
  h->es = L.es;
  h->pop_bytes = L.pop_bytes;
  h->base = static_cast<char*>(dev_buf);
  h->buf[0] = h->base + L.off_buf[0];
  h->buf[1] = h->base + L.off_buf[1];
  h->hdr_dev = reinterpret_cast<TableHeader*>(h->base + L.off_hdr);
  h->desc_dev = reinterpret_cast<LatticeDesc*>(h->base + L.off_desc);
  h->partials = reinterpret_cast<double*>(h->base + L.off_partials);
  if (p->diag_every > 0) {
    h->ustage = reinterpret_cast<float*>(h->base + L.off_ustage);
    h->mode_tab = reinterpret_cast<double*>(h->base + L.off_modetab);
  }
  h->history = reinterpret_cast<double*>(h->base + L.off_hist);
  h->last = reinterpret_cast<double*>(h->base + L.off_last);
  h->hist_count = reinterpret_cast<int64_t*>(h->base + L.off_count);
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->wall = false;
  for (int a = 0; a < h->D; ++a) h->wall = h->wall || p->bc[a] == ELBM_BC_BOUNCEBACK;
  h->force = p->force[0] != 0.0 || p->force[1] != 0.0 || (h->D == 3 && p->force[2] != 0.0);
  h->staged = use_staged(*p);
  h->kind = h->D == 2 ? kKindD2
                      : (h->staged ? kKindD3Staged : (p->collision == ELBM_COLLISION_MRT ? kKindD3Mrt : kKindD3));
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->event, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "elbm_create");
  }
  fill_desc(h);
  // per-axis factors e^{i k_a lam_a x} of the diagnostic mode (sample steps)
  std::vector<double> mtab;
  if (p->diag_every > 0) {
    fill_diag_args(h);
    if (h->c64.has_mode) {
      mtab.resize(2 * size_t(L.modetab_len));
      int64_t off = 0;
      for (int a = 0; a < h->D; ++a) {
        for (int64_t x = 0; x < p->n[a]; ++x) {
          const double ph = h->c64.mode_k[a] * (double(x) * h->c64.lam[a]);
          mtab[2 * (off + x)] = std::cos(ph);
          mtab[2 * (off + x) + 1] = std::sin(ph);
        }
        off += p->n[a];
      }
    }
  }
  TableHeader hdr{};
  hdr.count = 1;
  hdr.total_tiles = h->ntiles;
  e = hipMemcpyAsync(h->hdr_dev, &hdr, sizeof hdr, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h->desc_dev, &h->desc, sizeof h->desc, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->hist_count, 0, sizeof(int64_t), h->stream);
  if (e == hipSuccess && !mtab.empty())
    e = hipMemcpyAsync(h->mode_tab, mtab.data(), mtab.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
  // The padding of the direction arrays is never written by the kernels; it
  // starts (and stays) zero so that saved states are byte-identical whenever
  // the populations are.
  for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipMemsetAsync(h->buf[b], 0, h->pop_bytes, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    (void)hipEventDestroy(h->event);
    delete h;
    return hip_fail(e, "elbm_create upload");
  }
  *out = h;
  return ELBM_OK;
}

int32_t elbm_init(elbm_handle h, const double* rho, const double* u) {
  if (!h || !rho || !u) return fail(ELBM_EINVAL, "NULL argument");
  int32_t s = set_dev(h->device);
  if (s) return s;
  h->step = 0;
  const int D = h->D;
  const int64_t per = int64_t(h->pop_bytes / (size_t(D + 1) * sizeof(double)));
  double* stage = static_cast<double*>(h->buf[1]);
  for (int64_t c0 = 0; c0 < h->N; c0 += per) {
    const int64_t cnt = std::min(per, h->N - c0);
    HIPCHK(hipMemcpyAsync(stage, rho + c0, cnt * sizeof(double), hipMemcpyHostToDevice, h->stream));
    for (int a = 0; a < D; ++a)
      HIPCHK(hipMemcpyAsync(stage + (1 + a) * cnt, u + a * h->N + c0, cnt * sizeof(double), hipMemcpyHostToDevice,
                            h->stream));
    HIPCHK(launch_init(h->c64, stage, c0, cnt, h->buf[0], h->stream));
  }
  // the staging area was the other buffer: return it to zero (see elbm_create)
  HIPCHK(hipMemsetAsync(h->buf[1], 0, h->pop_bytes, h->stream));
  s = reset_history(h);
  if (s) return s;
  HIPCHK(hipStreamSynchronize(h->stream));
  return ELBM_OK;
}

int32_t elbm_step(elbm_handle h, int64_t nsteps) {
  if (!h) return fail(ELBM_EINVAL, "NULL handle");
  if (nsteps < 0) return fail(ELBM_EINVAL, "nsteps must be >= 0");
  int32_t s = set_dev(h->device);
  if (s) return s;
  const int grid = grid_for_tiles(h->ntiles);
  const int grid_diag = std::min(grid, kDiagBlocks);
  for (int64_t k = 0; k < nsteps; ++k) {
    const bool sample = h->p.diag_every > 0 && (h->step + 1) % h->p.diag_every == 0;
    if (sample) {
      // the sample step: the step kernel also forms the record's moments
      // (its tiles spread over at most kDiagBlocks blocks, one partial each)
      HIPCHK(launch_step_diag(h->kind, h->p.storage, h->wall, h->force, h->hdr_dev, h->desc_dev, h->step, grid_diag,
                              h->dargs, h->stream));
      HIPCHK(launch_diag_tail(h->c64, h->ustage, h->partials, grid_diag, h->history, h->hist_count,
                              int32_t(h->p.diag_capacity), h->last, h->step + 1, h->stream));
    } else {
      HIPCHK(launch_step(h->kind, h->p.storage, h->wall, h->force, h->hdr_dev, h->desc_dev, h->step, grid,
                         h->stream));
    }
    ++h->step;
  }
  return ELBM_OK;
}

int64_t elbm_step_count(elbm_handle h) { return h ? h->step : -1; }

int32_t elbm_kernel(elbm_handle h, elbm_kernel_info* out) {
  if (!h || !out) return fail(ELBM_EINVAL, "NULL argument");
  elbm_kernel_info k{};
  k.kernel = h->staged ? ELBM_KERNEL_STAGED : ELBM_KERNEL_REGISTER;
  k.block_threads = step_block_threads(h->kind);
  k.tile[0] = h->D == 3 ? (h->staged ? 64 : kTileX3) : 64 * kStrips2;
  k.tile[1] = h->D == 3 ? (h->staged ? kRowsStaged : kRows3) : 1;
  k.tile[2] = h->desc.chunk;
  k.blocks_per_cu = step_blocks_per_cu(h->kind, h->p.storage, h->wall, h->force);
  k.tiles = h->ntiles;
  *out = k;
  return ELBM_OK;
}

int32_t elbm_fields(elbm_handle h, double* rho, double* u) {
  if (!h || !rho || !u) return fail(ELBM_EINVAL, "NULL argument");
  int32_t s = set_dev(h->device);
  if (s) return s;
  double* stage = static_cast<double*>(spare_buf(h));
  for (int comp = 0; comp <= h->D; ++comp) {
    HIPCHK(launch_field(h->c64, state_buf(h), comp, stage, h->stream));
    double* dst = comp == 0 ? rho : u + int64_t(comp - 1) * h->N;
    HIPCHK(hipMemcpyAsync(dst, stage, h->N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return ELBM_OK;
}

int32_t elbm_populations(elbm_handle h, double* f) {
  if (!h || !f) return fail(ELBM_EINVAL, "NULL argument");
  int32_t s = set_dev(h->device);
  if (s) return s;
  double* stage = static_cast<double*>(spare_buf(h));
  for (int i = 0; i < h->Q; ++i) {
    HIPCHK(launch_pop_out(h->c64, state_buf(h), i, stage, h->stream));
    HIPCHK(hipMemcpyAsync(f + int64_t(i) * h->N, stage, h->N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return ELBM_OK;
}

int32_t elbm_set_populations(elbm_handle h, const double* f) {
  if (!h || !f) return fail(ELBM_EINVAL, "NULL argument");
  int32_t s = set_dev(h->device);
  if (s) return s;
  h->step = 0;
  double* stage = static_cast<double*>(h->buf[1]);
  for (int i = 0; i < h->Q; ++i) {
    HIPCHK(hipMemcpyAsync(stage, f + int64_t(i) * h->N, h->N * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCHK(launch_pop_in(h->c64, stage, i, h->buf[0], h->stream));
  }
  s = reset_history(h);
  if (s) return s;
  HIPCHK(hipStreamSynchronize(h->stream));
  return ELBM_OK;
}

int32_t elbm_diag(elbm_handle h, elbm_diag_record* out) {
  if (!h || !out) return fail(ELBM_EINVAL, "NULL argument");
  int32_t s = set_dev(h->device);
  if (s) return s;
  s = run_diag(h, false);
  if (s) return s;
  double rec[kRec];
  HIPCHK(hipMemcpyAsync(rec, h->last, sizeof rec, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  record_to_diag(rec, out);
  if (out->nan_count > 0 || !(out->min_rho > 0.0))
    return fail(ELBM_EUNSTABLE, "non-finite moment or non-positive density at step " + std::to_string(h->step));
  return ELBM_OK;
}

int32_t elbm_diag_history(elbm_handle h, elbm_diag_record* out, int32_t max, int32_t* count) {
  if (!h || !count || (max > 0 && !out)) return fail(ELBM_EINVAL, "NULL argument");
  *count = 0;
  const int32_t cap = h->p.diag_every > 0 ? h->p.diag_capacity : 0;
  if (cap == 0 || max <= 0) return ELBM_OK;
  int32_t s = set_dev(h->device);
  if (s) return s;
  int64_t n = 0;
  std::vector<double> ring(size_t(cap) * kRec);
  HIPCHK(hipMemcpyAsync(&n, h->hist_count, sizeof n, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(ring.data(), h->history, ring.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const int64_t kept = std::min<int64_t>(n, cap);
  const int64_t first = n - kept;
  const int64_t take = std::min<int64_t>(kept, max);
  for (int64_t r = 0; r < take; ++r) record_to_diag(&ring[size_t((first + r) % cap) * kRec], &out[r]);
  *count = int32_t(take);
  return ELBM_OK;
}

int32_t elbm_checkpoint_bytes(elbm_handle h, size_t* bytes) {
  if (!h || !bytes) return fail(ELBM_EINVAL, "NULL argument");
  *bytes = sizeof(CkptHeader) + size_t(h->nplanes) * size_t(h->Q) * size_t(h->pstride) * h->es;
  return ELBM_OK;
}

int32_t elbm_save(elbm_handle h, void* host, size_t bytes) {
  if (!h || !host) return fail(ELBM_EINVAL, "NULL argument");
  size_t need = 0;
  elbm_checkpoint_bytes(h, &need);
  if (bytes < need) return fail(ELBM_EINVAL, "checkpoint buffer too small");
  int32_t s = set_dev(h->device);
  if (s) return s;
  CkptHeader hd{};
  std::memcpy(hd.magic, kCkptMagic, 8);
  hd.abi = ELBM_ABI_VERSION;
  hd.es = uint32_t(h->es);
  hd.step = h->step;
  hd.pstride = h->pstride;
  hd.bytes = int64_t(need);
  hd.params = h->p;
  std::memcpy(host, &hd, sizeof hd);
  HIPCHK(hipMemcpyAsync(static_cast<char*>(host) + sizeof hd, state_buf(h), need - sizeof hd, hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return ELBM_OK;
}

int32_t elbm_load(elbm_handle h, const void* host, size_t bytes) {
  if (!h || !host) return fail(ELBM_EINVAL, "NULL argument");
  size_t need = 0;
  elbm_checkpoint_bytes(h, &need);
  if (bytes < need) return fail(ELBM_EINVAL, "checkpoint buffer too small");
  CkptHeader hd;
  std::memcpy(&hd, host, sizeof hd);
  if (std::memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.abi != ELBM_ABI_VERSION || hd.es != h->es ||
      hd.pstride != h->pstride || hd.bytes != int64_t(need) || !same_problem(hd.params, h->p) || hd.step < 0)
    return fail(ELBM_EINVAL, "checkpoint does not match this lattice");
  int32_t s = set_dev(h->device);
  if (s) return s;
  h->step = hd.step;
  HIPCHK(hipMemcpyAsync(state_buf(h), static_cast<const char*>(host) + sizeof hd, need - sizeof hd,
                        hipMemcpyHostToDevice, h->stream));
  s = reset_history(h);
  if (s) return s;
  HIPCHK(hipStreamSynchronize(h->stream));
  return ELBM_OK;
}

int32_t elbm_sync(elbm_handle h) {
  if (!h) return fail(ELBM_EINVAL, "NULL handle");
  int32_t s = set_dev(h->device);
  if (s) return s;
  HIPCHK(hipStreamSynchronize(h->stream));
  return ELBM_OK;
}

int32_t elbm_destroy(elbm_handle h) {
  if (!h) return ELBM_OK;
  set_dev(h->device);
  hipError_t e = hipStreamSynchronize(h->stream);
  (void)hipEventDestroy(h->event);
  delete h;
  if (e != hipSuccess) return hip_fail(e, "elbm_destroy");
  return ELBM_OK;
}

// ---------------------------------------------------------------- batches

int32_t elbm_batch_create(int32_t capacity, void* hip_stream, elbm_batch* out) {
  if (!out) return fail(ELBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (capacity < 1 || capacity > 65536) return fail(ELBM_EINVAL, "capacity must lie in [1, 65536]");
  auto* b = new (std::nothrow) elbm_batch_s();
  if (!b) return fail(ELBM_EINVAL, "out of host memory");
  b->capacity = capacity;
  b->caller = static_cast<hipStream_t>(hip_stream);
  const size_t tbytes = align_up(sizeof(TableHeader), 64) + size_t(capacity) * sizeof(LatticeDesc);
  hipError_t e = hipGetDevice(&b->device);
  // a stream of its own: the legacy default stream cannot be captured into a graph
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->host_stage), tbytes * kClasses);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->entry, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (b->host_stage) (void)hipHostFree(b->host_stage);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return hip_fail(e, "elbm_batch_create");
  }
  *out = b;
  return ELBM_OK;
}

int32_t elbm_batch_run(elbm_batch b, const elbm_handle* hs, const int64_t* steps, int32_t count, int32_t use_graph) {
  if (!b) return fail(ELBM_EINVAL, "NULL batch");
  if (count < 0 || count > b->capacity) return fail(ELBM_EINVAL, "count exceeds the batch capacity");
  if (count > 0 && (!hs || !steps)) return fail(ELBM_EINVAL, "NULL argument");
  for (int32_t k = 0; k < count; ++k) {
    if (!hs[k]) return fail(ELBM_EINVAL, "NULL handle in batch");
    if (steps[k] < 0) return fail(ELBM_EINVAL, "steps must be >= 0");
    if (hs[k]->device != b->device) return fail(ELBM_EINVAL, "lattice on another device");
    for (int32_t m = 0; m < k; ++m)
      if (hs[m] == hs[k]) return fail(ELBM_EINVAL, "a lattice appears twice in the batch");
  }
  int32_t s = set_dev(b->device);
  if (s) return s;
  int64_t smax = 0;
  for (int32_t k = 0; k < count; ++k) smax = std::max(smax, steps[k]);
  if (smax == 0) return ELBM_OK;

  const size_t hbytes = align_up(sizeof(TableHeader), 64);
  const size_t tbytes = hbytes + size_t(b->capacity) * sizeof(LatticeDesc);
  // the pinned staging must not change while the previous upload is pending
  if (b->copy_pending) HIPCHK(hipEventSynchronize(b->copied));

  // group by kernel class; within a class keep the caller's order
  std::vector<std::vector<int32_t>> members(kClasses);
  for (int32_t k = 0; k < count; ++k) {
    if (steps[k] == 0) continue;
    const elbm_lattice* h = hs[k];
    members[class_of(h->kind, h->p.storage, h->wall, h->force)].push_back(k);
  }
  uint64_t mask = 0;
  std::vector<int> grids;
  for (int c = 0; c < kClasses; ++c) {
    if (members[c].empty()) continue;
    mask |= uint64_t(1) << c;
    char* hostt = b->host_stage + size_t(c) * tbytes;
    auto* hdr = reinterpret_cast<TableHeader*>(hostt);
    auto* tab = reinterpret_cast<LatticeDesc*>(hostt + hbytes);
    int64_t base = 0;
    int n = 0;
    for (int32_t k : members[c]) {
      LatticeDesc d = hs[k]->desc;
      d.tile_base = base;
      d.parity0 = int32_t(hs[k]->step & 1);
      d.nsteps = steps[k];
      base += d.ntiles;
      tab[n++] = d;
    }
    hdr->count = n;
    hdr->pad = 0;
    hdr->total_tiles = base;
    if (!b->dev_tables.count(c)) {
      char* p = nullptr;
      HIPCHK(hipMalloc(reinterpret_cast<void**>(&p), tbytes));
      b->dev_tables[c] = p;
    }
    grids.push_back(batch_grid(base));
  }
  // order the device work after what is pending on the caller's and the lattices' streams
  HIPCHK(hipEventRecord(b->entry, b->caller));
  HIPCHK(hipStreamWaitEvent(b->stream, b->entry, 0));
  for (int32_t k = 0; k < count; ++k) {
    HIPCHK(hipEventRecord(hs[k]->event, hs[k]->stream));
    HIPCHK(hipStreamWaitEvent(b->stream, hs[k]->event, 0));
  }
  for (int c = 0; c < kClasses; ++c) {
    if (!(mask & (uint64_t(1) << c))) continue;
    const size_t n = hbytes + size_t(members[c].size()) * sizeof(LatticeDesc);
    HIPCHK(hipMemcpyAsync(b->dev_tables[c], b->host_stage + size_t(c) * tbytes, n, hipMemcpyHostToDevice, b->stream));
  }
  HIPCHK(hipEventRecord(b->copied, b->stream));
  b->copy_pending = true;

  auto launch_all = [&](hipStream_t st) -> int32_t {
    for (int64_t sub = 0; sub < smax; ++sub) {
      int gi = 0;
      for (int c = 0; c < kClasses; ++c) {
        if (!(mask & (uint64_t(1) << c))) continue;
        const ClassKey ck = class_key(c);
        const auto* hdr = reinterpret_cast<const TableHeader*>(b->dev_tables[c]);
        const auto* tab = reinterpret_cast<const LatticeDesc*>(b->dev_tables[c] + hbytes);
        HIPCHK(launch_step(ck.kind, ck.storage, ck.wall, ck.force, hdr, tab, sub, grids[gi++], st));
      }
    }
    return ELBM_OK;
  };

  if (use_graph) {
    auto key = std::make_tuple(mask, smax, grids);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
      HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      const int32_t ls = launch_all(b->stream);
      hipGraph_t graph = nullptr;
      const hipError_t ee = hipStreamEndCapture(b->stream, &graph);
      if (ls != ELBM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return ls;
      }
      if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
      hipGraphExec_t exec = nullptr;
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
      if (b->graphs.size() >= 64) {
        (void)hipGraphExecDestroy(b->graphs.begin()->second);
        b->graphs.erase(b->graphs.begin());
      }
      it = b->graphs.emplace(key, exec).first;
    }
    HIPCHK(hipGraphLaunch(it->second, b->stream));
  } else {
    s = launch_all(b->stream);
    if (s) return s;
  }
  HIPCHK(hipEventRecord(b->done, b->stream));
  HIPCHK(hipStreamWaitEvent(b->caller, b->done, 0));
  for (int32_t k = 0; k < count; ++k) {
    hs[k]->step += steps[k];
    HIPCHK(hipStreamWaitEvent(hs[k]->stream, b->done, 0));
  }
  return ELBM_OK;
}

int32_t elbm_batch_destroy(elbm_batch b) {
  if (!b) return ELBM_OK;
  set_dev(b->device);
  (void)hipStreamSynchronize(b->stream);
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : b->dev_tables) (void)hipFree(kv.second);
  if (b->host_stage) (void)hipHostFree(b->host_stage);
  (void)hipEventDestroy(b->copied);
  (void)hipEventDestroy(b->done);
  (void)hipEventDestroy(b->entry);
  (void)hipStreamDestroy(b->stream);
  delete b;
  return ELBM_OK;
}

// ------------------------------------------- allocation-free batched runs

int32_t elbm_batch_run_static(const elbm_handle* hs, const int64_t* steps, int32_t count, void* hip_stream) {
  if (count < 0 || count > kStaticMaxLattices)
    return fail(ELBM_EINVAL, "elbm_batch_run_static takes at most " + std::to_string(kStaticMaxLattices) +
                                 " lattices per call (" + std::to_string(count) + " given)");
  if (count == 0) return ELBM_OK;
  if (!hs || !steps) return fail(ELBM_EINVAL, "NULL argument");
  for (int32_t k = 0; k < count; ++k) {
    if (!hs[k]) return fail(ELBM_EINVAL, "NULL handle in batch");
    if (steps[k] < 0) return fail(ELBM_EINVAL, "steps must be >= 0");
    if (hs[k]->device != hs[0]->device) return fail(ELBM_EINVAL, "lattices on different devices");
    for (int32_t m = 0; m < k; ++m)
      if (hs[m] == hs[k]) return fail(ELBM_EINVAL, "a lattice appears twice in the batch");
  }
  int32_t s = set_dev(hs[0]->device);
  if (s) return s;
  int64_t smax = 0;
  for (int32_t k = 0; k < count; ++k) smax = std::max(smax, steps[k]);
  if (smax == 0) return ELBM_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  void* scr = nullptr;
  HIPCHK(static_scratch(&scr));  // first call on this device: looks the address up

  // Table image (host, fixed size): class headers, then the descriptors of
  // every class in class order, each class in the caller's order.
  thread_local unsigned char image[kStaticScratchBytes];
  auto* hdrs = reinterpret_cast<TableHeader*>(image);
  auto* descs = reinterpret_cast<LatticeDesc*>(image + kStaticHeaderBytes);
  int32_t first[kClasses], ncls[kClasses];
  int64_t tiles[kClasses];
  int32_t order[kStaticMaxLattices];
  for (int c = 0; c < kClasses; ++c) ncls[c] = 0, tiles[c] = 0;
  for (int32_t k = 0; k < count; ++k)
    if (steps[k] > 0) {
      const elbm_lattice* h = hs[k];
      ++ncls[class_of(h->kind, h->p.storage, h->wall, h->force)];
    }
  int32_t used = 0;
  for (int c = 0; c < kClasses; ++c) {
    first[c] = used;
    used += ncls[c];
    ncls[c] = 0;
  }
  for (int32_t k = 0; k < count; ++k) {
    if (steps[k] == 0) continue;
    const elbm_lattice* h = hs[k];
    const int c = class_of(h->kind, h->p.storage, h->wall, h->force);
    order[first[c] + ncls[c]++] = k;
  }
  for (int c = 0; c < kClasses; ++c) {
    for (int32_t m = 0; m < ncls[c]; ++m) {
      const int32_t k = order[first[c] + m];
      LatticeDesc d = hs[k]->desc;
      d.tile_base = tiles[c];
      d.parity0 = int32_t(hs[k]->step & 1);
      d.nsteps = steps[k];
      tiles[c] += d.ntiles;
      descs[first[c] + m] = d;
    }
    hdrs[c] = TableHeader{ncls[c], 0, tiles[c]};
  }
  const size_t bytes = kStaticHeaderBytes + size_t(used) * sizeof(LatticeDesc);

  // order after the work queued on the lattices' streams
  for (int32_t k = 0; k < count; ++k) {
    HIPCHK(hipEventRecord(hs[k]->event, hs[k]->stream));
    HIPCHK(hipStreamWaitEvent(st, hs[k]->event, 0));
  }
  HIPCHK(launch_write_bytes(scr, image, bytes, st));
  auto* dhdr = static_cast<const TableHeader*>(scr);
  auto* dtab = reinterpret_cast<const LatticeDesc*>(static_cast<const unsigned char*>(scr) + kStaticHeaderBytes);
  for (int64_t sub = 0; sub < smax; ++sub)
    for (int c = 0; c < kClasses; ++c) {
      if (ncls[c] == 0) continue;
      const ClassKey ck = class_key(c);
      HIPCHK(launch_step(ck.kind, ck.storage, ck.wall, ck.force, dhdr + c, dtab + first[c], sub,
                         batch_grid(tiles[c]), st));
    }
  // the lattices' streams wait for the run
  for (int32_t k = 0; k < count; ++k) {
    hs[k]->step += steps[k];
    HIPCHK(hipEventRecord(hs[k]->event, st));
    HIPCHK(hipStreamWaitEvent(hs[k]->stream, hs[k]->event, 0));
  }
  return ELBM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- open faces

struct elbm_faces_s {
  elbm_lattice* h = nullptr;
  int D = 2;
  FaceArgs args{};      // D2Q9 open faces
  Walls3Args args3{};   // D3Q27 Grad walls on the y faces
};

namespace {

struct FacePlan {
  std::vector<FaceNode> nodes;  // boundary nodes on one face, then corner nodes
  int32_t n_single = 0, n_corner = 0;
  std::vector<FaceGhost> ghosts;
  int32_t o[2] = {0, 0}, n[2] = {0, 0};
  size_t off_nodes = 0, off_ghosts = 0, off_mom = 0, bytes = 0;
};

bool face_odd(int kind) { return kind == ELBM_FACE_SYMMETRY || kind == ELBM_FACE_WALL; }

// D3Q27: Grad walls on both y faces, x and z periodic; the storage carries one
// ghost row below and one above the fluid. Device bytes: the wall nodes'
// pulled (rho, j_y), then their inward neighbours' velocities.
int32_t plan_walls3(const elbm_lattice* h, const elbm_faces_params* fp, size_t& bytes) {
  if (h->p.u_adv[0] != 0.0 || h->p.u_adv[1] != 0.0 || h->p.u_adv[2] != 0.0)
    return fail(ELBM_EUNSUPPORTED, "Grad walls need u_adv == 0 (rest reference)");
  for (int a = 0; a < 3; ++a)
    if (h->p.bc[a] != ELBM_BC_PERIODIC)
      return fail(ELBM_EINVAL, "the lattice under Grad walls is periodic (bc); the walls replace its bounce-back");
  if (fp->kind[0] != ELBM_FACE_PERIODIC || fp->kind[1] != ELBM_FACE_PERIODIC || fp->kind[2] != ELBM_FACE_WALL ||
      fp->kind[3] != ELBM_FACE_WALL)
    return fail(ELBM_EUNSUPPORTED, "D3Q27 lattices take Grad walls on both y faces with x (and z) periodic");
  for (int F = 0; F < 4; ++F)
    if (fp->node_kind[F]) return fail(ELBM_EUNSUPPORTED, "D3Q27 walls take one kind per face (node_kind NULL)");
  if (h->p.n[1] < 5) return fail(ELBM_EINVAL, "n_y must be the fluid rows (>= 3) plus 2 ghost rows");
  if (!std::isfinite(fp->wall_velocity[2]) || !std::isfinite(fp->wall_velocity[3]))
    return fail(ELBM_EINVAL, "wall velocities must be finite");
  const size_t nodes = size_t(2) * size_t(h->p.n[0]) * size_t(h->p.n[2]);
  bytes = align_up(nodes * 2 * sizeof(double), kAlign) + align_up(nodes * 3 * sizeof(double), kAlign);
  return ELBM_OK;
}

int32_t plan_faces(const elbm_lattice* h, const elbm_faces_params* fp, FacePlan& P) {
  if (!h || !fp) return fail(ELBM_EINVAL, "NULL argument");
  if (fp->abi_version != ELBM_ABI_VERSION) return fail(ELBM_EINVAL, "faces abi_version mismatch");
  if (h->D != 2) return fail(ELBM_EUNSUPPORTED, "open faces are implemented for D2Q9 lattices only");
  if (h->p.u_adv[0] != 0.0 || h->p.u_adv[1] != 0.0)
    return fail(ELBM_EUNSUPPORTED, "open faces need u_adv == 0 (rest reference)");
  if (h->p.bc[0] != ELBM_BC_PERIODIC || h->p.bc[1] != ELBM_BC_PERIODIC)
    return fail(ELBM_EINVAL, "the lattice under open faces is periodic (bc); the faces replace its walls");
  for (int F = 0; F < 4; ++F) {
    if (fp->kind[F] < ELBM_FACE_PERIODIC || fp->kind[F] > ELBM_FACE_OUTLET)
      return fail(ELBM_EINVAL, "face kind out of range");
    if (fp->kind[F] == ELBM_FACE_PERIODIC && fp->node_kind[F])
      return fail(ELBM_EINVAL, "a periodic face takes no per-node kinds");
  }
  for (int a = 0; a < 2; ++a) {
    const bool plo = fp->kind[2 * a] == ELBM_FACE_PERIODIC, phi = fp->kind[2 * a + 1] == ELBM_FACE_PERIODIC;
    if (plo != phi) return fail(ELBM_EINVAL, "a periodic axis is periodic on both faces");
    P.o[a] = plo ? 0 : 1;
    P.n[a] = int32_t(h->p.n[a]) - 2 * P.o[a];
    if (P.o[a] && P.n[a] < 3)
      return fail(ELBM_EINVAL, "an open axis needs >= 3 fluid nodes (lattice extent = fluid + 2 ghost nodes)");
  }
  // kinds per face node
  std::vector<int> kinds[4];
  for (int F = 0; F < 4; ++F) {
    const int m = F < 2 ? P.n[1] : P.n[0];
    kinds[F].assign(m, fp->kind[F]);
    if (fp->node_kind[F])
      for (int t = 0; t < m; ++t) {
        const int k = fp->node_kind[F][t];
        if (k < ELBM_FACE_SYMMETRY || k > ELBM_FACE_OUTLET)
          return fail(ELBM_EINVAL, "per-node face kinds are SYMMETRY, WALL, INLET or OUTLET");
        kinds[F][t] = k;
      }
  }
  for (int F = 0; F < 4; ++F) {
    bool outlet = false;
    for (int k : kinds[F]) outlet = outlet || k == ELBM_FACE_OUTLET;
    if (outlet && !(fp->outlet_density[F] > 0.0 && std::isfinite(fp->outlet_density[F])))
      return fail(ELBM_EINVAL, "an OUTLET face needs a positive, finite outlet_density");
    for (int b = 0; b < 2; ++b)
      if (!std::isfinite(fp->inlet_velocity[F][b])) return fail(ELBM_EINVAL, "inlet_velocity must be finite");
    if (!std::isfinite(fp->wall_velocity[F])) return fail(ELBM_EINVAL, "wall_velocity must be finite");
  }
  // boundary nodes (fluid coordinates)
  std::map<std::pair<int, int>, int> index;
  const int nx = P.n[0], ny = P.n[1];
  auto on = [&](int F, int x, int y) {
    if (!P.o[F >> 1]) return false;
    return (F == 0 && x == 0) || (F == 1 && x == nx - 1) || (F == 2 && y == 0) || (F == 3 && y == ny - 1);
  };
  std::vector<FaceNode> corners;
  for (int F = 0; F < 4; ++F) {
    if (!P.o[F >> 1]) continue;
    const int m = F < 2 ? ny : nx;
    for (int t = 0; t < m; ++t) {
      const int x = F < 2 ? (F == 0 ? 0 : nx - 1) : t, y = F < 2 ? t : (F == 2 ? 0 : ny - 1);
      int nf = 0;
      for (int G = 0; G < 4; ++G) nf += on(G, x, y) ? 1 : 0;
      if (nf == 1) {
        index[{x, y}] = int(P.nodes.size());
        P.nodes.push_back(FaceNode{x, y, F, kinds[F][t]});
      } else if (F < 2) {
        const int k = kinds[F][t];
        if (k != ELBM_FACE_INLET && k != ELBM_FACE_OUTLET)
          return fail(ELBM_EUNSUPPORTED, "a corner node needs an INLET or OUTLET x face");
        corners.push_back(FaceNode{x, y, F, k});
      }
    }
  }
  P.n_single = int32_t(P.nodes.size());
  for (const FaceNode& c : corners) {
    index[{c.x, c.y}] = int(P.nodes.size());
    P.nodes.push_back(c);
  }
  P.n_corner = int32_t(corners.size());
  // ghost ring (storage coordinates)
  const int NX = int(h->p.n[0]), NY = int(h->p.n[1]);
  for (int Y = 0; Y < NY; ++Y)
    for (int X = 0; X < NX; ++X) {
      const bool gx = P.o[0] && (X == 0 || X == NX - 1), gy = P.o[1] && (Y == 0 || Y == NY - 1);
      if (!gx && !gy) continue;
      FaceGhost g{X, Y, -1, 0, 1.0};
      if (gx != gy) {
        const int a = gx ? 0 : 1;
        const int x = X - P.o[0], y = Y - P.o[1];
        const int fx = gx ? (X == 0 ? 0 : nx - 1) : x, fy = gy ? (Y == 0 ? 0 : ny - 1) : y;
        const int F = gx ? (X == 0 ? 0 : 1) : (Y == 0 ? 2 : 3);
        const int t = a == 0 ? fy : fx;
        g.node = index.at({fx, fy});
        g.axis = a;
        g.parity = face_odd(kinds[F][t]) ? -1.0 : 1.0;
      }
      P.ghosts.push_back(g);
    }
  P.off_nodes = 0;
  P.off_ghosts = align_up(P.nodes.size() * sizeof(FaceNode), kAlign);
  P.off_mom = P.off_ghosts + align_up(P.ghosts.size() * sizeof(FaceGhost), kAlign);
  P.bytes = P.off_mom + align_up(P.nodes.size() * 3 * sizeof(double), kAlign) + kAlign;
  return ELBM_OK;
}

}  // namespace

extern "C" {

int32_t elbm_faces_query_bytes(elbm_handle lattice, const elbm_faces_params* fp, size_t* bytes) {
  if (!bytes) return fail(ELBM_EINVAL, "NULL argument");
  if (lattice && fp && lattice->D == 3) {
    if (fp->abi_version != ELBM_ABI_VERSION) return fail(ELBM_EINVAL, "faces abi_version mismatch");
    return plan_walls3(lattice, fp, *bytes);
  }
  FacePlan P;
  const int32_t s = plan_faces(lattice, fp, P);
  if (s) return s;
  *bytes = P.bytes;
  return ELBM_OK;
}

int32_t elbm_faces_create(elbm_handle h, const elbm_faces_params* fp, void* dev_buf, size_t bytes,
                          elbm_faces_handle* out) {
  if (!out) return fail(ELBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (h && fp && h->D == 3) {
    if (fp->abi_version != ELBM_ABI_VERSION) return fail(ELBM_EINVAL, "faces abi_version mismatch");
    size_t need = 0;
    int32_t s3 = plan_walls3(h, fp, need);
    if (s3) return s3;
    if (!dev_buf) return fail(ELBM_EINVAL, "dev_buf is NULL");
    if (reinterpret_cast<uintptr_t>(dev_buf) % kAlign) return fail(ELBM_EINVAL, "dev_buf must be 256-byte aligned");
    if (bytes < need)
      return fail(ELBM_ENOMEM, "device buffer holds " + std::to_string(bytes) + " bytes, " + std::to_string(need) +
                                   " needed");
    auto* f = new (std::nothrow) elbm_faces_s();
    if (!f) return fail(ELBM_EINVAL, "out of host memory");
    f->h = h;
    f->D = 3;
    Walls3Args& A = f->args3;
    A.pstride = h->pstride;
    A.storage = h->p.storage;
    A.scale = h->c64.scale;
    A.inv_scale = h->c64.inv_scale;
    for (int a = 0; a < 3; ++a) {
      A.N[a] = int32_t(h->p.n[a]);
      A.n[a] = int32_t(h->p.n[a]) - (a == 1 ? 2 : 0);
      A.lam[a] = h->p.lambda[a];
      A.g[a] = h->p.force[a];
    }
    A.T = h->p.T;
    A.omega = h->p.omega;
    A.omega_bulk = h->p.collision == ELBM_COLLISION_MRT ? h->p.omega_bulk : h->p.omega;
    for (int i = 0; i < 27; ++i) A.w[i] = h->c64.W[0][i % 3] * h->c64.W[1][(i / 3) % 3] * h->c64.W[2][i / 9];
    A.wall_u[0] = fp->wall_velocity[2];
    A.wall_u[1] = fp->wall_velocity[3];
    A.mom = static_cast<double*>(dev_buf);
    A.uin = reinterpret_cast<double*>(static_cast<char*>(dev_buf) +
                                      align_up(size_t(2) * size_t(A.n[0]) * size_t(A.n[2]) * 2 * sizeof(double), kAlign));
    *out = f;
    return ELBM_OK;
  }
  FacePlan P;
  int32_t s = plan_faces(h, fp, P);
  if (s) return s;
  if (!dev_buf) return fail(ELBM_EINVAL, "dev_buf is NULL");
  if (reinterpret_cast<uintptr_t>(dev_buf) % kAlign) return fail(ELBM_EINVAL, "dev_buf must be 256-byte aligned");
  if (bytes < P.bytes)
    return fail(ELBM_ENOMEM, "device buffer holds " + std::to_string(bytes) + " bytes, " + std::to_string(P.bytes) +
                                 " needed");
  s = set_dev(h->device);
  if (s) return s;
  char* base = static_cast<char*>(dev_buf);
  if (!P.nodes.empty())
    HIPCHK(hipMemcpyAsync(base + P.off_nodes, P.nodes.data(), P.nodes.size() * sizeof(FaceNode),
                          hipMemcpyHostToDevice, h->stream));
  if (!P.ghosts.empty())
    HIPCHK(hipMemcpyAsync(base + P.off_ghosts, P.ghosts.data(), P.ghosts.size() * sizeof(FaceGhost),
                          hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  auto* f = new (std::nothrow) elbm_faces_s();
  if (!f) return fail(ELBM_EINVAL, "out of host memory");
  f->h = h;
  FaceArgs& A = f->args;
  A.pstride = h->pstride;
  A.storage = h->p.storage;
  A.scale = h->c64.scale;
  A.inv_scale = h->c64.inv_scale;
  for (int a = 0; a < 2; ++a) {
    A.N[a] = int32_t(h->p.n[a]);
    A.o[a] = P.o[a];
    A.n[a] = P.n[a];
    A.lam[a] = h->p.lambda[a];
    A.g[a] = h->p.force[a];
  }
  A.T = h->p.T;
  A.omega = h->p.omega;
  A.omega_bulk = h->p.collision == ELBM_COLLISION_MRT ? h->p.omega_bulk : h->p.omega;
  for (int i = 0; i < 9; ++i) A.w[i] = h->c64.W[0][i % 3] * h->c64.W[1][i / 3];
  for (int F = 0; F < 4; ++F) {
    A.wall_u[F] = fp->wall_velocity[F];
    A.inlet_u[F][0] = fp->inlet_velocity[F][0];
    A.inlet_u[F][1] = fp->inlet_velocity[F][1];
    A.outlet_rho[F] = fp->outlet_density[F];
  }
  A.nodes = reinterpret_cast<const FaceNode*>(base + P.off_nodes);
  A.n_single = P.n_single;
  A.n_corner = P.n_corner;
  A.ghosts = reinterpret_cast<const FaceGhost*>(base + P.off_ghosts);
  A.n_ghost = int32_t(P.ghosts.size());
  A.mom = reinterpret_cast<double*>(base + P.off_mom);
  *out = f;
  return ELBM_OK;
}

int32_t elbm_faces_step(elbm_faces_handle f, int64_t nsteps) {
  if (!f) return fail(ELBM_EINVAL, "NULL handle");
  if (nsteps < 0) return fail(ELBM_EINVAL, "nsteps must be >= 0");
  elbm_lattice* h = f->h;
  int32_t s = set_dev(h->device);
  if (s) return s;
  for (int64_t k = 0; k < nsteps; ++k) {
    if (f->D == 3) {
      f->args3.h = state_buf(h);
      HIPCHK(launch_walls3(f->args3, h->stream));
    } else {
      f->args.h = state_buf(h);
      HIPCHK(launch_faces(f->args, h->stream));
    }
    s = elbm_step(h, 1);
    if (s) return s;
  }
  return ELBM_OK;
}

int32_t elbm_faces_destroy(elbm_faces_handle f) {
  delete f;
  return ELBM_OK;
}

}  // extern "C"
