// Internal declarations shared by the HIP kernels and the C-ABI host code.
//
// Axis roles inside the kernels. The kernels see three internal axes:
//   axis 0 -- x, the fastest (coalesced) axis, tiled in 64-wide wavefronts;
//   axis 1 -- the tiled row axis (y for D3Q27; absent, extent 1, for D2Q9);
//   axis 2 -- the marched axis, walked plane by plane with a register ring
//             (z for D3Q27; y for D2Q9).
// So a D2Q9 lattice n_x x n_y is handled as internal extents (n_x, 1, n_y)
// with velocity components (c_x, 0, c_y).
//
// Population layout ("plane slabs"). The state is stored plane by plane along
// the marched axis: plane z holds Q arrays, one per direction, each covering
// the plane's n_0 n_1 nodes x fastest and padded to `pstride` elements; so
// population i of the node with in-plane index p on plane z sits at element
//   z * Q * pstride + i * pstride + p.
// Every offset inside one slab (Q pstride elements) stays below 2^32 bytes, so
// the step kernel addresses a slab through one buffer resource with 32-bit
// offsets, whatever the size of the whole lattice.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace elbm {

#ifndef ELBM_TX3
#define ELBM_TX3 64
#endif
#ifndef ELBM_TY3
#define ELBM_TY3 8
#endif
#ifndef ELBM_TYS
#define ELBM_TYS 16
#endif
constexpr int kTileX3 = ELBM_TX3;  // x width of a D3Q27 tile
constexpr int kRows3 = ELBM_TY3;   // y rows of a D3Q27 tile
constexpr int kRowsStaged = ELBM_TYS;     // y rows of a tile of the LDS-staged kernel (x width 64)
constexpr int kStrips2 = 4;        // 64-wide strips of a D2Q9 tile -> 256 threads
constexpr int kDiagBlocks = 1024;  // fixed grid of the diagnostic reductions
constexpr int kRec = 16;           // doubles per diagnostic record / partial
constexpr float kF16Scale = 4096.0f;

// Record layout (doubles) of a diagnostic partial or history entry.
enum RecField {
  R_STEP = 0, R_MASS, R_MOM0, R_MOM1, R_MOM2, R_KE, R_ENS, R_MODE_RE, R_MODE_IM,
  R_MAXU, R_MINRHO, R_NAN, R_USED
};

// One entry of the device descriptor table: everything a block needs to
// advance one tile of one lattice. Plain data, copied host -> device.
struct alignas(16) LatticeDesc {
  void* buf[2];            // population buffers; state of substep s is in buf[(parity0 + s) & 1]
  int64_t pstride;         // elements between consecutive direction arrays of a plane slab
  int64_t tile_base;       // first global tile index of this lattice in its table
  int64_t ntiles;          // tiles of this lattice
  int64_t nsteps;          // substeps this lattice takes part in (s < nsteps)
  int32_t n[3];            // internal extents (see axis roles above)
  int32_t tiles[3];        // tile counts along the internal axes
  int32_t chunk;           // marched planes per tile
  int32_t parity0;
  int32_t wall[3];         // internal axis has halfway bounce-back walls
  int32_t pad0;
  float lam[3];            // stretching per internal axis (1 on an absent axis)
  float inv_lam[3];
  float inv_lam2[3];
  float half_inv_lam[3];   // 1 / (2 lambda): central-difference factor
  float mfac[3];           // lambda / scale: stored-value sums -> momentum deviation
  float anom[3];           // lambda^2 - 3T: linear coefficient of the anomaly
  float uref[3];           // reference velocity of the stored deviations
  float W[3][3];           // reference triplets Psi_c(uref, T + uref^2, lambda), c = -1, 0, 1
  float WW[3][3];          // W[0][c0] * W[1][c1] (rounded from FP64)
  float g[3];              // body-force acceleration
  float T;
  float omega;
  float coef;              // (2 - omega)/(2 omega); 0 for the uncorrected control
  float om1;               // 1 - omega
  float oms;               // omega * scale
  float inv_scale;         // stored value * inv_scale = deviation
  float scale;
  int32_t mrt;             // D2Q9 multi-relaxation-time collision
  float om1g;              // 1 - omega_ghost
  float cdev;              // omega_ghost - omega
  float ciso;              // omega_ghost - omega_bulk
  float coefb;             // (2 - omega_bulk)/(2 omega_bulk); 0 for the uncorrected control
  float one;               // 1.0, read at run time (see Puller::line_moments)
  float pad1[2];
};

struct TableHeader {
  int32_t count;
  int32_t pad;
  int64_t total_tiles;
};

// FP64 constants of a lattice used by the (non-hot) conversion, init and
// diagnostic kernels.
struct LatticeConst64 {
  int32_t D, Q;
  int32_t n[3];            // physical extents (x, y, z), z = 1 for D2Q9
  int32_t wall[3];         // physical axes
  int64_t pstride;         // elements between direction arrays of a plane slab
  int64_t plane;           // nodes per plane of the marched axis (n_x n_y; n_x for D2Q9)
  int64_t N;
  double lam[3];           // physical axes
  double T;
  double uref[3];
  double g[3];
  double W[3][3];          // physical axes, reference triplets
  double scale, inv_scale;
  double mode_k[3];
  double mode_dir[3];
  int32_t storage;
  int32_t has_mode;
};

// Diagnostics folded into a step (sample steps of elbm_step): the step kernel
// forms, per node, rho and the reported velocity u = j/rho + g/2 of its pulled
// (post-streaming) populations in FP64. These are the moments of the step's
// post-collision state at that node (the collision conserves rho and adds the
// force impulse rho g to j, so j/rho + g/2 = j'/rho - g/2). The kernel
// accumulates the FP64 sums of a diagnostic record per block (partials, fields
// other than the enstrophy) and stages u in FP32 for the enstrophy pass.
struct DiagArgs {
  float* ustage;           // 3 N floats, component-major over the physical axes, node order x fastest
  double* partials;        // kRec doubles per block of the launch
  const double* mode_tab;  // (cos, sin) of mode_k[a] lam[a] x for x < n[a], axis a at mode_tab + 2 mode_off[a]
  double lam[3];           // physical axes
  double uref[3];
  double g[3];
  double mode_dir[3];
  double inv_scale;
  int64_t N;
  int32_t n[3];            // physical extents
  int32_t mode_off[3];
  int32_t has_mode;
};

// ---- allocation-free batched runner (elbm_static.hip) ----
constexpr int kStaticMaxLattices = 256;   // lattices per elbm_batch_run_static call
constexpr int kStaticClasses = 48;        // kernel classes (one table each)
constexpr size_t kStaticHeaderBytes = 1024;  // kStaticClasses TableHeaders, padded
constexpr size_t kStaticScratchBytes = kStaticHeaderBytes + size_t(kStaticMaxLattices) * sizeof(LatticeDesc);
static_assert(sizeof(LatticeDesc) == 336, "the static scratch size the header documents (1024 + 336 per lattice)");
static_assert(kStaticClasses * sizeof(TableHeader) <= kStaticHeaderBytes, "table headers fit");
static_assert(kStaticHeaderBytes % alignof(LatticeDesc) == 0, "descriptors stay aligned");
// Device address of the fixed scratch array on the current device (looked up
// once per device and kept).
hipError_t static_scratch(void** out);
// Writes `bytes` host bytes to device memory `dst` with kernels on `st` (the
// bytes travel as kernel arguments: no staging memory).
hipError_t launch_write_bytes(void* dst, const unsigned char* src, size_t bytes, hipStream_t st);

// ---- open boundaries of a D2Q9 lattice (elbm_faces.hip) ----
// A fluid boundary node (fluid coordinates) with the face it is on
// (0: x-, 1: x+, 2: y-, 3: y+) and that face's kind at it (ELBM_FACE_*).
struct FaceNode {
  int32_t x, y;
  int32_t face, kind;
};
// A ghost node (storage coordinates), the boundary node whose anomaly it
// mirrors across the face (index into the node list, -1 for none: corner
// ghosts), the face's normal axis and the parity of the mirrored normal
// momentum (-1 at walls and symmetry planes, +1 at inlets and outlets).
struct FaceGhost {
  int32_t X, Y;
  int32_t node, axis;
  double parity;
};
struct FaceArgs {
  void* h;                // state buffer (deviations in storage format), plane slabs along y
  int64_t pstride;
  int32_t storage;        // ELBM_STORE_F32 / F16 / BF16
  int32_t spad;
  double scale, inv_scale;  // stored value = scale x deviation
  int32_t N[2];           // storage extents (fluid + ghost ring on open axes)
  int32_t o[2];           // 1 on an open axis (ghost ring), 0 on a periodic one
  int32_t n[2];           // fluid extents
  double lam[2], T, omega, g[2];
  double omega_bulk;      // trace rate of the MRT collision (omega under LBGK)
  double w[9];            // reference weights of the deviations
  double wall_u[4];       // tangential wall velocity per face
  double inlet_u[4][2];   // inlet velocity per face
  double outlet_rho[4];   // outlet density per face
  const FaceNode* nodes;  // n_single boundary nodes on one face, then n_corner corner nodes
  int32_t n_single, n_corner;
  const FaceGhost* ghosts;
  int32_t n_ghost, pad;
  double* mom;            // 3 doubles per node: pulled rho, j_x, j_y after the fill
};
// Rewrites the ghost ring of the state for the next pull (boundary nodes on
// one face, then corners, then the ghosts' anomaly populations).
hipError_t launch_faces(const FaceArgs& a, hipStream_t st);

// Grad's-approximation walls on the y faces of a D3Q27 lattice (x and z
// periodic): the storage carries one ghost row below and one above the fluid.
struct Walls3Args {
  void* h;                // state buffer (deviations in storage format), plane slabs along z
  int64_t pstride;
  int32_t storage;        // ELBM_STORE_F32 / F16 / BF16
  int32_t pad;
  double scale, inv_scale;  // stored value = scale x deviation
  int32_t N[3];           // storage extents (n_y + 2 rows)
  int32_t n[3];           // fluid extents
  double lam[3], T, omega, omega_bulk, g[3];
  double w[27];           // reference weights of the deviations
  double wall_u[2];       // x-velocity of the low and the high wall
  double* mom;            // 2 doubles per wall node (pulled rho, j_y), low face then high face
  double* uin;            // 3 doubles per wall node: velocity of its inward neighbour
};
hipError_t launch_walls3(const Walls3Args& a, hipStream_t st);

// ---- launchers (defined in the .hip translation units) ----
// Step kernel families: the D2Q9 register-pull kernel (LBGK, or the
// multi-relaxation-time collision as a runtime branch), the D3Q27
// register-pull kernel, the LDS-staged D3Q27 kernel for 16-bit storage
// (periodic x and z, full tiles), and the D3Q27 register-pull kernel with the
// multi-relaxation-time collision (a variant of its own: the LBGK kernel's
// registers are not shared with it).
enum StepKind : int { kKindD2 = 0, kKindD3 = 1, kKindD3Staged = 2, kKindD3Mrt = 3 };
constexpr int kKinds = 4;
hipError_t launch_step(int kind, int storage, bool wall, bool force, const TableHeader* hdr,
                       const LatticeDesc* table, int64_t substep, int grid, hipStream_t st);
// The same step with the diagnostics of its post-collision state folded in
// (one lattice per table; grid at most kDiagBlocks blocks, one partial record
// per block).
hipError_t launch_step_diag(int kind, int storage, bool wall, bool force, const TableHeader* hdr,
                            const LatticeDesc* table, int64_t substep, int grid, const DiagArgs& da,
                            hipStream_t st);
int step_block_threads(int kind);
// Resident step blocks per compute unit for a kernel class (occupancy query).
int step_blocks_per_cu(int kind, int storage, bool wall, bool force);

hipError_t launch_init(const LatticeConst64& c, const double* stage, int64_t cell0, int64_t count,
                       void* dst, hipStream_t st);
hipError_t launch_pop_out(const LatticeConst64& c, const void* src, int i, double* out, hipStream_t st);
hipError_t launch_pop_in(const LatticeConst64& c, const double* in, int i, void* dst, hipStream_t st);
hipError_t launch_field(const LatticeConst64& c, const void* src, int comp, double* out, hipStream_t st);
// Diagnostics of the state in `src`: the record goes to `last`, and is also
// appended to the ring `history` (capacity records, count in *hist_count)
// when capacity > 0. `ustage` holds 3 N floats of scratch; `partials` 2
// kDiagBlocks records (the moment sums, then the enstrophy sums).
hipError_t launch_diag(const LatticeConst64& c, const void* src, float* ustage, double* partials,
                       double* history, int64_t* hist_count, int32_t capacity, double* last,
                       int64_t step, hipStream_t st);
// After a step with folded diagnostics (launch_step_diag, nb_moments partial
// records in `partials`): the enstrophy pass over the staged velocity and the
// final fixed-order reduction into `last` and the history.
hipError_t launch_diag_tail(const LatticeConst64& c, const float* ustage, double* partials, int nb_moments,
                            double* history, int64_t* hist_count, int32_t capacity, double* last, int64_t step,
                            hipStream_t st);

}  // namespace elbm
