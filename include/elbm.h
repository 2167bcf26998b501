/*
 * elbm.h -- C ABI of the extended lattice Boltzmann (LBGK) step library for
 * AMD MI355X (gfx950).
 *
 * The library advances lattices of populations with the LBGK equation of
 * Saadat, Dorschner and Karlin, "Extended Lattice Boltzmann Model"
 * (arXiv:2101.04550): pull streaming, moments, the diagonal third-moment
 * anomaly, its central difference, the extended diagonal pressure, the
 * product-form equilibrium and relaxation (Sec. 2.1-2.4), on the D2Q9 and
 * D3Q27 tensor-product velocity sets with per-axis stretching (Sec. 2.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an elbm_status (0 = ELBM_OK); no C++ exception
 *   crosses this boundary. On failure, elbm_last_error() returns a
 *   thread-local message describing the most recent error of this thread.
 * - Units: gas constant R = 1, time step 1 (Sec. 3). A population with
 *   c_ia = +-1 moves one node per step; its velocity is lambda_a c_ia
 *   (Sec. 2.2), so lambda_a is the node spacing along axis a.
 * - Node order: cell index = x + n_x (y + n_y z) (x fastest). For D2Q9,
 *   n_z = 1 and cell = x + n_x y.
 * - Velocity order: i = sum_a (c_ia + 1) 3^a over the axes of the lattice,
 *   c_ia in {-1, 0, 1}; the opposite of direction i is Q - 1 - i.
 * - Host arrays are borrowed for the duration of the call only. Device
 *   memory passed to elbm_create is caller-owned and borrowed until
 *   elbm_destroy. Handles are library-owned.
 * - One handle may be used by one thread at a time. Work is queued on the
 *   HIP stream given at creation; calls that return host data synchronise
 *   that stream.
 */
#ifndef ELBM_H
#define ELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ELBM_ABI_VERSION 2u

typedef enum elbm_status {
  ELBM_OK = 0,
  ELBM_EINVAL = 1,        /* a parameter is out of range or inconsistent      */
  ELBM_EUNSUPPORTED = 2,  /* valid request the library does not implement    */
  ELBM_ENOMEM = 3,        /* the device buffer is smaller than required       */
  ELBM_EDEVICE = 4,       /* a HIP runtime call failed (text in last_error)   */
  ELBM_EUNSTABLE = 5      /* diagnostics saw a non-finite value or rho <= 0   */
} elbm_status;

enum { ELBM_BC_PERIODIC = 0, ELBM_BC_BOUNCEBACK = 1 };

enum { ELBM_COLLISION_BGK = 0, ELBM_COLLISION_MRT = 1 };

/* Storage of the populations in device memory. The kernels always compute
 * in FP32 on deviations h_i = f_i - w_i from the reference equilibrium
 * w_i = f^eq_i(rho = 1, u_adv) (the lattice weights when u_adv = 0).
 * ELBM_STORE_F32 keeps h_i in FP32; F16 and BF16 keep h_i * 2^12 (F16) or
 * h_i (BF16), rounded to nearest even. */
enum { ELBM_STORE_F32 = 0, ELBM_STORE_F16 = 1, ELBM_STORE_BF16 = 2 };

/* Problem statement of one lattice (Sec. 2 and Sec. 3 of the paper).
 *  abi_version  must equal ELBM_ABI_VERSION.
 *  lattice      9 (D2Q9) or 27 (D3Q27) (Sec. 2.2, tensor-product velocity set).
 *  n[3]         node extents along x, y, z; D2Q9 requires n[2] == 1.
 *  lambda[3]    stretching factors lambda_a > 0 (Sec. 2.2, stretched velocities);
 *               lambda[2] is ignored for D2Q9.
 *  T            temperature (R = 1) (Sec. 2.1).
 *  omega        relaxation parameter in (0, 2); kinematic viscosity
 *               nu = (1/omega - 1/2) T (Sec. 2.1, eq. nu).
 *  u_adv[3]     advection velocity added to the initial velocity field by
 *               elbm_init, and reference velocity of the stored deviations;
 *               must be 0 on a lattice with bounce-back walls
 *               (ELBM_EUNSUPPORTED otherwise).
 *  force[3]     constant body-force acceleration g (Sec. 3.5), applied by the
 *               exact-difference method F_i = f^eq_i(rho, u + g) - f^eq_i(rho, u).
 *  bc[3]        per axis ELBM_BC_PERIODIC or ELBM_BC_BOUNCEBACK (halfway
 *               bounce-back walls on both faces of that axis).
 *  storage      ELBM_STORE_F32 / ELBM_STORE_F16 / ELBM_STORE_BF16.
 *  extended     1: extended equilibrium (Sec. 2.3, eq. 27eqext);
 *               0: uncorrected product-form equilibrium (Sec. 2.3, eq. 27eq).
 *  diag_every   0: no automatic diagnostics; k > 0: elbm_step records the
 *               diagnostics of every k-th step into a device-resident history
 *               (formed by that step's own kernel; needs 12 bytes per node
 *               more device memory, see elbm_query_bytes).
 *  diag_capacity number of history records kept (ring buffer), >= 1 when
 *               diag_every > 0.
 *  mode_k[3]    physical wave vector k of the measured plane mode, and
 *  mode_dir[3]  the velocity direction d whose amplitude
 *               < (d.u) exp(-i k.x) > the diagnostics report (Sec. 3.1).
 *  collision    ELBM_COLLISION_BGK (Sec. 2.1, eq. LBGK) or ELBM_COLLISION_MRT
 *               (the multi-relaxation-time extension that Sec. 4 names; D3Q27
 *               lattices with it take the register-pull kernel, never the
 *               LDS-staged one): the deviatoric non-equilibrium stress relaxes at
 *               omega, its trace at omega_bulk, the non-equilibrium part
 *               above second order at omega_ghost (the stress parts mapped
 *               back by the linear Grad map of the product-form lattice),
 *               and the pressure correction of Sec. 2.4 takes the bulk
 *               rate's factor (2 - omega_bulk)/(2 omega_bulk) on its
 *               isotropic part. Shear viscosity nu = (1/omega - 1/2) T;
 *               sound decays by (nu + (1/omega_bulk - 1/2) T) k^2 / 2.
 *  omega_bulk, omega_ghost  in (0, 2) when collision is MRT, else unused.
 */
typedef struct elbm_params {
  uint32_t abi_version;
  int32_t lattice;
  int64_t n[3];
  double lambda[3];
  double T;
  double omega;
  double u_adv[3];
  double force[3];
  int32_t bc[3];
  int32_t storage;
  int32_t extended;
  int32_t diag_every;
  int32_t diag_capacity;
  int32_t collision;
  double mode_k[3];
  double mode_dir[3];
  double omega_bulk;
  double omega_ghost;
} elbm_params;

/* Global diagnostics of the post-collision state after `step` steps, reduced
 * in FP64 (Sec. 3.1-3.3). The reported velocity is u = (j + rho g/2)/rho
 * with j the pre-force momentum.
 *  mass       sum over nodes of rho
 *  mom[3]     sum over nodes of rho u
 *  ke         (1/2) <u.u>                    (volume average, Sec. 3.2)
 *  enstrophy  <|curl u|^2>, central differences with spacing lambda_a
 *             (Sec. 3.3); no-slip ghost u(-1) = -u(0) on wall axes
 *  mode_re, mode_im   <(d.u) exp(-i k.x)>, x_a = node index * lambda_a
 *  max_uperp  max over nodes of |d.u|         (Sec. 3.1)
 *  min_rho    minimum density
 *  nan_count  number of nodes holding a non-finite moment */
typedef struct elbm_diag_record {
  int64_t step;
  double mass;
  double mom[3];
  double ke;
  double enstrophy;
  double mode_re;
  double mode_im;
  double max_uperp;
  double min_rho;
  int64_t nan_count;
} elbm_diag_record;

/* How the library advances a lattice (inspection and measurement). */
enum { ELBM_KERNEL_REGISTER = 0, ELBM_KERNEL_STAGED = 1 };
typedef struct elbm_kernel_info {
  int32_t kernel;         /* ELBM_KERNEL_REGISTER: each node pulls its Q values
                             with one load apiece; ELBM_KERNEL_STAGED: a block
                             stages the rows its tile pulls from in LDS (D3Q27
                             LBGK, 16-bit storage, n_x % 64 == 0, x and z
                             periodic, y bounce-back with n_y % 16 == 0 or
                             periodic with n_y > 8) */
  int32_t block_threads;  /* threads per workgroup */
  int32_t tile[3];        /* tile extent along the internal axes: x, y (1 for
                             D2Q9), and the planes marched per tile */
  int32_t blocks_per_cu;  /* resident workgroups per compute unit */
  int64_t tiles;          /* tiles per step (workgroup tasks) */
} elbm_kernel_info;

typedef struct elbm_lattice* elbm_handle;
typedef struct elbm_batch_s* elbm_batch;

/* Version of the ABI this library implements (ELBM_ABI_VERSION). */
uint32_t elbm_abi_version(void);

/* Human-readable name of a status code. Never NULL; static storage. */
const char* elbm_status_string(int32_t status);

/* Thread-local text of the last error raised on this thread ("" if none). */
const char* elbm_last_error(void);

/* Checks a parameter set without touching the GPU (Sec. 2.1: omega in (0,2),
 * T > 0; Sec. 2.2: lambda > 0, rest-population weight 1 - T/lambda^2 > 0 on
 * every axis; at least 3 nodes on a periodic axis, 2 on a wall axis; at most
 * 2^31 - 1 nodes, and Q times the nodes of one plane across the slowest axis
 * (n_x n_y for D3Q27, n_x for D2Q9) times the element size below 2^32 bytes).
 * Returns ELBM_EINVAL or ELBM_EUNSUPPORTED (bounce-back walls together with a
 * nonzero u_adv) with a message, else ELBM_OK. */
int32_t elbm_validate(const elbm_params* params);

/* Device bytes a lattice needs: two population buffers (ping-pong) of about
 * Q * N * sizeof(storage) bytes each (stored plane by plane along the slowest
 * axis, each direction's array of a plane padded to 64 elements) plus a small
 * fixed scratch area (descriptor, diagnostic partial sums, history; with
 * diag_every > 0 also 3 N floats of staged velocity and 16 bytes per node of
 * each axis for the mode factors). Pure host arithmetic. */
int32_t elbm_query_bytes(const elbm_params* params, size_t* bytes);

/* Creates a lattice in the caller's device buffer `dev_buf` of `bytes`
 * bytes (>= elbm_query_bytes, 256-byte aligned; ELBM_ENOMEM if smaller) on
 * the current HIP device. `hip_stream` (a hipStream_t, may be NULL for the
 * null stream) is borrowed. The populations are left undefined until
 * elbm_init or elbm_set_populations. `*out` receives the handle. */
int32_t elbm_create(const elbm_params* params, void* dev_buf, size_t bytes,
                    void* hip_stream, elbm_handle* out);

/* Initial post-collision state f'_i(x, 0) = f^eq_i(rho, u + u_adv) with the
 * equilibrium pressure P^eq = T + u^2 (Sec. 2.3, eq. 27eq); the step count
 * is reset to 0 and the diagnostic history cleared.
 *  rho  host FP64 array of N = n_x n_y n_z densities (node order above)
 *  u    host FP64 array of D * N velocities, component-major: u[a * N + cell]
 * Synchronises the stream before returning. */
int32_t elbm_init(elbm_handle h, const double* rho, const double* u);

/* Advances the lattice by `nsteps` >= 0 LBGK steps (Sec. 2.1, eq. LBGK):
 * per step one fused kernel that pulls, computes moments and the anomaly,
 * its central difference (Sec. 2.3, eq. Paastar1), the extended pressure,
 * the product form and relaxes (plus the force). Asynchronous on the
 * handle's stream. If diag_every > 0, every diag_every-th step runs the
 * same kernel with the diagnostics folded in: it sums the FP64 moments of
 * the pulled populations of each node, which are the moments of the node's
 * post-collision state (the collision conserves rho and adds rho g to j), so
 * the record equals elbm_diag of that state up to the rounding of the stored
 * values; the record is appended to the history. The state after such a step
 * is bitwise the state without diagnostics. */
int32_t elbm_step(elbm_handle h, int64_t nsteps);

/* Number of steps taken since elbm_init / elbm_set_populations. */
int64_t elbm_step_count(elbm_handle h);

/* The step kernel and launch shape chosen for this lattice (fixed at
 * elbm_create). Two environment variables read at elbm_create override the
 * choice, for measurements: ELBM_STAGED=0 forces the register kernel, and
 * ELBM_CHUNK=c (an integer >= 1) sets the planes marched per tile (capped at
 * the lattice's extent along that axis; every value gives the same results).
 * ELBM_EINVAL on NULL arguments. Host only. */
int32_t elbm_kernel(elbm_handle h, elbm_kernel_info* out);

/* Macroscopic fields of the current state, FP64, host arrays owned by the
 * caller: rho[N], u[D * N] (component-major), u = (j + rho g/2)/rho.
 * Synchronises. */
int32_t elbm_fields(elbm_handle h, double* rho, double* u);

/* Populations of the current (post-collision) state as FP64 f_i = w_i + h_i:
 * f[i * N + cell], Q * N values. Synchronises. */
int32_t elbm_populations(elbm_handle h, double* f);

/* Replaces the current state with the FP64 populations f[i * N + cell]
 * (converted to the storage format, deviations rounded to nearest even),
 * resets the step count and clears the history. Synchronises. */
int32_t elbm_set_populations(elbm_handle h, const double* f);

/* Computes the diagnostics of the current (stored) state now, by a pass that
 * reads it. Synchronises.
 * Returns ELBM_EUNSTABLE (with *out filled) if a node holds a non-finite
 * moment or rho <= 0. */
int32_t elbm_diag(elbm_handle h, elbm_diag_record* out);

/* Copies up to `max` recorded diagnostics, oldest first, into `out`;
 * `*count` receives the number copied. Synchronises. */
int32_t elbm_diag_history(elbm_handle h, elbm_diag_record* out, int32_t max, int32_t* count);

/* Bytes of a checkpoint of this lattice (populations + step count). */
int32_t elbm_checkpoint_bytes(elbm_handle h, size_t* bytes);

/* Copies the state (raw stored populations and the step count) into the host
 * buffer `host` of `bytes` >= elbm_checkpoint_bytes bytes. Synchronises. */
int32_t elbm_save(elbm_handle h, void* host, size_t bytes);

/* Restores a state written by elbm_save for a lattice with identical
 * parameters; the run continues bitwise as if it had not been interrupted.
 * ELBM_EINVAL if the checkpoint does not match. Synchronises. */
int32_t elbm_load(elbm_handle h, const void* host, size_t bytes);

/* Waits for all work queued on the handle's stream. */
int32_t elbm_sync(elbm_handle h);

/* Releases the handle (not the caller's device buffer). Synchronises. */
int32_t elbm_destroy(elbm_handle h);

/* ---- batched fused launches (many resident lattices, one launch per class) ----
 *
 * A batch owns a device descriptor table for up to `capacity` lattices and a
 * cache of captured HIP graphs. elbm_batch_run advances lattice hs[k] by
 * steps[k] >= 0 steps: every step is one launch per class of lattices
 * (lattice, storage, walls, force) over all their tiles, whatever their
 * sizes; lattices that have taken their steps sit out the remaining
 * launches. Each lattice advances bitwise exactly as under elbm_step.
 * With use_graph != 0 the launch sequence of the longest run is captured
 * once into a HIP graph (cached by that length) and replayed; the table is
 * uploaded before each replay. Automatic diagnostics are not recorded in a
 * batch run. All lattices must live on the batch's device; none may appear
 * twice. The batch allocates its own device memory, pinned host staging and
 * a non-blocking stream (library-owned); `hip_stream` (may be NULL) is only
 * used for ordering: a run starts after the work queued on it and on the
 * lattices' streams, and they wait for the run's end. */
int32_t elbm_batch_create(int32_t capacity, void* hip_stream, elbm_batch* out);
int32_t elbm_batch_run(elbm_batch b, const elbm_handle* hs, const int64_t* steps,
                       int32_t count, int32_t use_graph);
int32_t elbm_batch_destroy(elbm_batch b);

/* ---- the same batched run for callers that cannot allocate ----
 *
 * For callers that must not allocate device or pinned host memory: code that
 * runs between allocation-free phases of a serving loop, harnesses that forbid
 * hipMalloc, streams being captured into a graph by the caller. Advances
 * lattice hs[k] by steps[k] >= 0 steps exactly as elbm_batch_run (same
 * kernels, same results bitwise), with no batch object: the per-class
 * descriptor tables live in a fixed device array that the library holds on
 * every device it runs on until the process ends (1024 + 336 *
 * ELBM_STATIC_MAX_LATTICES bytes); they are written by small kernels whose
 * arguments carry the bytes. Nothing is allocated and no graph is captured.
 *  hs, steps   count lattices (all on the current device, none twice) and
 *              their step counts; count <= ELBM_STATIC_MAX_LATTICES, else
 *              ELBM_EINVAL.
 *  hip_stream  the stream the run is queued on (may be NULL); it first waits
 *              for the work queued on the lattices' streams, and they wait
 *              for the run's end.
 * Every call on a device rewrites the one table array of that device: calls
 * whose runs overlap on one device (different streams, no ordering between
 * them) race and must not be made. Automatic diagnostics are not recorded. */
#define ELBM_STATIC_MAX_LATTICES 256
int32_t elbm_batch_run_static(const elbm_handle* hs, const int64_t* steps, int32_t count, void* hip_stream);

/* ---- Open boundaries of a D2Q9 lattice ----
 * The paper's wall-bounded cases use Grad's approximation for the walls
 * (Sec. 3, opening paragraph, after a cited reference that it does not
 * restate); its flat plate (Sec. 3.4) also needs an inlet, an outlet and a
 * symmetry plane. The faces below implement one reading of these (stated in
 * full in csrc/elbm_faces.hip); each face of the fluid rectangle has a kind
 * per face node:
 *  ELBM_FACE_PERIODIC  the axis is periodic (both faces, every node)
 *  ELBM_FACE_SYMMETRY  free-slip plane halfway outside the boundary row
 *                      (specular reflection)
 *  ELBM_FACE_WALL      no-slip wall halfway outside the boundary row, moving
 *                      tangentially at wall_velocity[f]; the populations
 *                      entering from the wall are Grad's approximation at a
 *                      velocity interpolated through the wall, the density
 *                      of the node's mass and normal-momentum balance and
 *                      the Navier-Stokes stress of the interpolated velocity
 *                      (with the MRT collision: its trace part at
 *                      omega_bulk; with omega_bulk != omega the wall then
 *                      misses the bulk's second-order normal stresses and
 *                      exchanges mass with the flow at that order)
 *  ELBM_FACE_INLET     prescribed velocity inlet_velocity[f] at the halfway
 *                      plane (bounce-back from a surface moving at it)
 *  ELBM_FACE_OUTLET    prescribed density outlet_density[f], with the inward
 *                      neighbour's velocity and non-equilibrium part
 * Faces are indexed 0: x-, 1: x+, 2: y-, 3: y+. A corner node (on two
 * non-periodic faces) follows its x face, which must then be INLET or
 * OUTLET. */
enum {
  ELBM_FACE_PERIODIC = 0,
  ELBM_FACE_SYMMETRY = 1,
  ELBM_FACE_WALL = 2,
  ELBM_FACE_INLET = 3,
  ELBM_FACE_OUTLET = 4
};

/*  abi_version     ELBM_ABI_VERSION
 *  kind[4]         kind of every node of face f, unless node_kind[f] is set
 *  node_kind[4]    NULL or a host array of one kind per fluid node along
 *                  face f (n_y for x faces, n_x for y faces; read at create)
 *  wall_velocity   tangential velocity of the WALL nodes of face f
 *  inlet_velocity  (u_x, u_y) of the INLET nodes of face f
 *  outlet_density  density of the OUTLET nodes of face f (> 0 where used) */
typedef struct elbm_faces_params {
  uint32_t abi_version;
  int32_t kind[4];
  const int8_t* node_kind[4];
  double wall_velocity[4];
  double inlet_velocity[4][2];
  double outlet_density[4];
} elbm_faces_params;

typedef struct elbm_faces_s* elbm_faces_handle;

/* Device bytes of the face tables of `lattice` (node lists, ghost list,
 * per-node moments). The lattice must be D2Q9 (any storage: FP16 / BF16
 * face values are rounded to the storage format like any stored value), u_adv = 0
 * and both axes periodic (bc), and it must carry the ghost ring: its
 * extents are the fluid extents plus 2 along every axis whose faces are not
 * PERIODIC (fluid extents >= 3 there). A D3Q27 lattice takes the faces of a
 * channel: PERIODIC x faces, WALL y faces (one kind per face, node_kind
 * NULL; wall_velocity[2], [3]: the x-velocity of the low and the high wall),
 * z periodic, any storage (FP16 / BF16: the wall populations are rounded
 * to the storage format like any stored value), u_adv = 0, all axes
 * periodic in bc and n_y the fluid rows (>= 3) plus 2 ghost rows. ELBM_EINVAL / ELBM_EUNSUPPORTED with
 * a message otherwise. Host arithmetic only. */
int32_t elbm_faces_query_bytes(elbm_handle lattice, const elbm_faces_params* fp, size_t* bytes);

/* Attaches the faces to `lattice`, with their tables in the caller's device
 * buffer (>= elbm_faces_query_bytes, 256-byte aligned); uploads on the
 * lattice's stream and synchronises. The lattice must outlive the handle. */
int32_t elbm_faces_create(elbm_handle lattice, const elbm_faces_params* fp, void* dev_buf, size_t bytes,
                          elbm_faces_handle* out);

/* Advances the lattice by nsteps steps, each preceded by the face update of
 * the ghost ring (three small kernels on the lattice's stream), as
 * elbm_step does otherwise (diagnostic samples included; they and
 * elbm_fields cover the ghost ring too). Asynchronous. */
int32_t elbm_faces_step(elbm_faces_handle f, int64_t nsteps);

/* Releases the host handle (the device buffer stays the caller's). */
int32_t elbm_faces_destroy(elbm_faces_handle f);

#ifdef __cplusplus
}
#endif

#endif /* ELBM_H */
