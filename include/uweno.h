/*
 * uweno — third-order WENO finite-volume residual on unstructured
 * quadrilateral, triangular and mixed meshes, for MI355X (gfx950).
 *
 * Method: Zhao, Pan, Wang, "A third-order WENO scheme on unstructured
 * quadrilateral and triangular meshes" (arXiv:1712.08317).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns uw_status; UW_OK == 0.  No C++ exception crosses the
 *   ABI.  On failure uw_last_error() returns a message for the calling
 *   thread, valid until that thread's next uw_* call.
 * - Cell numbering: uw_mesh_upload renumbers cells (quadrilaterals first,
 *   then triangles, each group along an order-16 Hilbert curve through the
 *   cells' vertex averages, ties by original id).  All device state arrays
 *   use this internal numbering; uw_mesh_info exports the permutation.
 * - State layout: device, structure of arrays W[v * n_cells + i], v the
 *   conserved variable (advection: 1 variable u; Euler: rho, rho u, rho v,
 *   rho E as in Sec. 2 of the paper), FP64, owned by the caller.
 * - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream).  Device work is enqueued asynchronously; device-side failures
 *   (non-finite values, non-positive density or pressure) are reported by
 *   uw_check, which synchronises the stream.
 * - Ownership: host inputs are borrowed for the duration of the call and
 *   copied; device tables belong to the mesh until uw_mesh_destroy.
 * - Concurrency: different meshes and batches may be used from different
 *   threads at once; calls on one mesh, or on one batch, must not overlap:
 *   they share its work buffers, captured graphs and error flag.  Device
 *   work on one mesh or batch queued on different streams must be ordered
 *   by the caller for the same reason.
 */
#ifndef UWENO_H
#define UWENO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  UW_OK = 0,
  UW_EINVAL = 1,      /* null pointer, bad size or enum value                    */
  UW_EMESH = 2,       /* invalid mesh (see uw_mesh_upload)                       */
  UW_ESTATE = 3,      /* call out of order (e.g. residual before precompute)     */
  UW_ENOMEM = 4,      /* host or device allocation failed                        */
  UW_EDEVICE = 5,     /* HIP error; the message names the call                   */
  UW_ENONFINITE = 6   /* device flagged NaN/Inf or rho <= 0 / p <= 0             */
} uw_status;

enum {
  UW_BC_PERIODIC = 0,
  UW_BC_TRANSMISSIVE = 1,
  UW_BC_REFLECTIVE = 2,
  UW_BC_INFLOW = 3,
  UW_BC_FRONT = 1 << 16
};
enum { UW_WENO = 0, UW_LINEAR = 1 };
enum { UW_CONSERVED = 0, UW_CHARACTERISTIC = 1 };
enum { UW_D_PER_GP = 0, UW_D_PER_CELL = 1 };
enum { UW_ADVECTION = 0, UW_EULER = 1 };
enum { UW_FP64 = 0, UW_FP32 = 1 };   /* UW_FP32: FP32 arithmetic, FP64 state */

typedef struct uw_mesh uw_mesh;
typedef struct uw_batch uw_batch;

/* Mesh description (host memory, borrowed for the call).
 * node_xy     [n_nodes][2] coordinates.
 * cell_nodes  [n_cells][4] counter-clockwise node indices; a triangle puts -1
 *             in slot 3.
 * node_id     [n_nodes] canonical node ids identifying periodic seam
 *             duplicates (duplicates sit exactly one period apart); NULL
 *             means every node is its own id.
 * bc          what an unmatched face is: UW_BC_TRANSMISSIVE (a mirrored ghost
 *             cell carrying the interior value), or UW_BC_PERIODIC (no
 *             unmatched face allowed).
 * face_bc     [n_cells][4] per-face kind of the unmatched faces, NULL = `bc`
 *             for all; entries of matched faces are ignored.  0 = `bc`,
 *             UW_BC_TRANSMISSIVE, UW_BC_REFLECTIVE (slip wall: the ghost and
 *             the outside state of the face flux are the inner state with its
 *             normal momentum reversed; transmissive for scalar advection),
 *             UW_BC_INFLOW + s (prescribed conserved state s of inflow_W),
 *             UW_BC_FRONT + f (moving front f of `fronts`).
 *             The paper's tests name non-reflecting, reflective and
 *             prescribed-state boundaries (Sec. 4) without defining them;
 *             the double Mach reflection's top boundary follows the exact
 *             motion of its shock, which a moving front describes.
 * n_inflow, inflow_W  number (<= 65533) and values [n_inflow][4] (rho,
 *             rho u, rho v, rho E; advection uses the first) of the
 *             prescribed states.
 * n_fronts, fronts  number (<= 2^20) and rows [n_fronts][12] = (ex, ey, c0,
 *             s, A[4], B[4]) of the moving fronts: at time t the outside
 *             state of a front face is state A if e.m < c0 + s t, m the
 *             face's midpoint (the mean of its two nodes as given), else
 *             state B.  Inside a Runge-Kutta step from t with step dt the
 *             three stages see the times t, t + dt and t + dt/2; e.m is
 *             formed in FP64 without fused multiply-adds, as is c0 + s t.
 * Errors: an unmatched face whose kind is UW_BC_PERIODIC gives UW_EMESH; a
 * kind outside the list, an inflow index >= n_inflow or a front index >=
 * n_fronts gives UW_EINVAL. */
typedef struct {
  int64_t n_nodes;
  const double* node_xy;
  int64_t n_cells;
  const int32_t* cell_nodes;
  const int32_t* node_id;
  int32_t bc;
  const int32_t* face_bc;
  int32_t n_inflow;
  const double* inflow_W;
  int32_t n_fronts;
  const double* fronts;
} uw_mesh_desc;

/* Scheme constants (paper Sec. 3): zeta of eq. (quadratic-2) (1e-14), theta
 * of the weight split of Sec. 3.4 (3; it must exceed 1: at 1 the negative
 * part of an all-positive weight set is empty), eps of the nonlinear weights (not
 * given by the paper; 1e-3), optimize = apply the linear-weight optimisation
 * of Sec. 3.3 (1), d_scope = UW_D_PER_GP (weights d from each Gauss point's
 * own linear weights) or UW_D_PER_CELL, mode = UW_WENO or UW_LINEAR (the
 * quadratic P^2 of eq. (polynomial-eta) at the Gauss points), variables =
 * UW_CONSERVED (component-wise) or UW_CHARACTERISTIC (Euler only; Sec. 4:
 * WENO on the characteristic variables of Roe's mean matrix between the
 * cell and the neighbour across each face, projected back; ignored for
 * scalar advection and in UW_LINEAR mode).  Any other value: UW_EINVAL.
 * theta is built into the tables by uw_precompute_geometry. */
typedef struct {
  double zeta, theta, eps;
  int32_t optimize, d_scope, mode, variables;
} uw_scheme;

/* Physics: equation = UW_ADVECTION (u_t + ax u_x + ay u_y = 0, upwind flux)
 * or UW_EULER (2D Euler, eq. (hyperbolic), HLLC flux, ratio `gamma`);
 * precision = UW_FP64 or UW_FP32.  UW_FP32 reconstructs and evaluates the
 * flux in FP32 (reciprocals, divisions and square roots with the hardware's
 * 1-ulp instructions) and keeps the state, the residual gather and the RK
 * stages in FP64; UW_FP64 does everything in FP64 (the reconstruction's
 * reciprocals as the hardware's refined by two Newton steps, the flux's
 * divisions and square roots correctly rounded). */
typedef struct {
  int32_t equation;
  double ax, ay, gamma;
  int32_t precision;
} uw_physics;

/* Precompute diagnostics (Sec. 3.3): largest |gamma| before/after the
 * optimisation, largest ||B gamma - eta||_inf and |sum gamma - 1| of the
 * optimised weights, number of absent stencil slots (E_j = 0), number of
 * cells whose big-stencil matrix A has rank < 5. */
typedef struct {
  double max_abs_gamma_raw, max_abs_gamma_opt, resid_opt, sum_dev;
  int64_t n_absent_slots, n_rank_deficient;
} uw_diag;

const char* uw_last_error(void);

/* Validates the mesh, builds face connectivity (periodic shifts, boundary
 * faces), the Hilbert renumbering and the big stencils (Sec. 3.1 quad
 * selection with substitutions i_j -> i_0, i_j -> i_{j-4}; Sec. 3.2
 * triangle selection with i_j -> i_0, i_j -> i_{j-3}), and binds the mesh
 * to HIP device `device`.  device = -1 builds a host-only mesh: connectivity,
 * stencils and the FP64 precompute can be inspected (uw_mesh_export,
 * uw_mesh_table) but every device call returns UW_ESTATE.
 * Errors: UW_EINVAL (null pointers, sizes < 1), UW_EMESH (a cell whose node
 * list is not 3 or 4 valid distinct nodes, signed area <= 0, an edge with
 * more than two owners or traversed twice in the same direction, an
 * unmatched face on a periodic mesh), UW_EDEVICE, UW_ENOMEM. */
uw_status uw_mesh_upload(const uw_mesh_desc* desc, int device, uw_mesh** out);

/* Sizes and the permutation.  new_of_old (nullable, host [n_cells]) receives
 * the internal index of every original cell. */
uw_status uw_mesh_info(const uw_mesh* mesh, int64_t* n_cells, int64_t* n_quads,
                       int64_t* n_interior_faces, int32_t* new_of_old);

/* Host export of the integer tables, internal numbering, for inspection.
 * slots   [n_cells][13]: the cell read by stencil slot j (after substitution;
 *         a ghost reads the cell itself; triangles use slots 0..9).
 * present [n_cells][13]: E_j.
 * nbr     [n_cells][4]: face neighbour (-1 boundary or unused slot).
 * Any pointer may be NULL. */
uw_status uw_mesh_export(const uw_mesh* mesh, int32_t* slots, uint8_t* present, int32_t* nbr);

/* FP64 precompute (Sec. 3.1-3.3): scaled-frame geometry, the regularised
 * least squares of eq. (quadratic-2) for eta (eq. (polynomial-eta)), the
 * candidate operators, B and the linear weights of eq.
 * (linearweight-matrix), the optimisation of Sec. 3.3.  Runs on the mesh's
 * GPU (one thread per cell) or, for a host-only mesh, on host threads, with
 * the same per-cell code.  The per-precision device tables are uploaded on
 * first use; a repeated call first waits for the device to finish the work
 * queued with the old tables, and drops the captured steps.  `diag` is
 * nullable.
 * Errors: UW_ESTATE (mesh not uploaded), UW_EINVAL, UW_ENOMEM, UW_EDEVICE. */
uw_status uw_precompute_geometry(uw_mesh* mesh, const uw_scheme* scheme, uw_diag* diag);

/* Host export of one FP64 table for inspection (internal numbering).
 * which: 0 = gamma [n][8][12], 1 = eta [n][8][13], 2 = candidate operators
 * Y [n][12][4], 3 = Gauss-point offsets [n][8][2], 4 = face normals and
 * scale [n][4][3] (nx, ny, |l|/(2|Omega|)), 5 = gamma before optimisation
 * [n][8][12].  Unused entries (triangles) are 0. */
uw_status uw_mesh_table(const uw_mesh* mesh, int32_t which, double* out);

/* L(W) of eq. (semidiscrete): L[v*n + i] = -(1/|Omega_i|) sum_p |l_p| sum_k
 * (1/2) F(x_pk).n_p, with WENO (or linear) face states at the Gauss points
 * of eq. (quadrature).  W, L: device FP64 [V][n_cells] (internal order).
 * Errors: UW_ESTATE (no precompute), UW_EINVAL, UW_EDEVICE. */
uw_status uw_residual(uw_mesh* mesh, const uw_physics* physics, const double* W, double* L,
                      void* stream);

/* uw_residual for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * It computes the same L(W) with the same kernels (bit for bit equal to
 * uw_residual) and calls no hipMalloc, hipFree or other allocating routine.
 * W, L: device FP64 [V][n_cells] (internal order), as for uw_residual;
 * owned by the caller.  Preconditions (else UW_ESTATE, nothing launched):
 * the mesh is precomputed and its device tables in physics->precision
 * exist, i.e. an earlier uw_residual, uw_residual_at, uw_rk3_step,
 * uw_cfl_dt or uw_autotune call in that precision ran on this mesh.
 * Scratch: the Gauss-point face states live in one fixed 64 MiB device
 * array per GPU, held from the library's load until the process ends;
 * n_cells * 8 * V * (4 in FP32, 8 in FP64) bytes must fit, i.e. at most
 * 524288 cells for FP32 Euler, 262144 for FP64 Euler, 2097152 and 1048576
 * for scalar advection; a larger mesh gets UW_EINVAL before any launch.
 * Every call on one GPU uses that GPU's array: calls whose execution
 * overlaps on the device (different streams, concurrent host threads)
 * race and give wrong results; calls ordered on one stream are safe.  No
 * value of the array needs to start at zero: each call writes every face
 * state it reads.  Device-side failures set the mesh's error flag
 * (uw_check).  Errors: UW_EINVAL, UW_ESTATE, UW_EDEVICE. */
uw_status uw_residual_noalloc(uw_mesh* mesh, const uw_physics* physics, const double* W,
                              double* L, void* stream);

/* uw_residual at time t (host value): only moving-front faces depend on
 * it; uw_residual is this call at t = 0. */
uw_status uw_residual_at(uw_mesh* mesh, const uw_physics* physics, const double* W, double* L,
                         double t, void* stream);

/* One step of the three-stage TVD Runge-Kutta scheme (Sec. 4), in place on
 * W.  t_dev: device double holding the time; dt = min(dt_fixed, t_end - t)
 * if dt_fixed > 0, else min(cfl * min_i 2|Omega_i| / sum_p |l_p|(|u.n_p| + c),
 * t_end - t); t_dev is advanced by dt on the device.  No host sync.  The
 * first call with a given (W, t_dev, cfl, dt_fixed, t_end, physics) captures
 * the step's launches into a hipGraph and later calls replay it (the null
 * stream is served by a library stream ordered with it); while per-kernel
 * timing is on (uw_profile) the launches are issued one by one instead.
 * At most 8 graphs are kept per mesh or batch: a new argument set beyond
 * that first waits for the device, then drops the least recently used one.
 * uw_precompute_geometry, uw_autotune, uw_schedule and uw_tile_size drop
 * the graphs (after the device has finished). */
uw_status uw_rk3_step(uw_mesh* mesh, const uw_physics* physics, double* W, double cfl,
                      double dt_fixed, double t_end, double* t_dev, void* stream);

/* n_steps (>= 0) steps of uw_rk3_step in one call, captured together (the
 * graph key adds n_steps).  Inside the run, the last stage of each step
 * also forms the next step's CFL bound from the state it writes (the same
 * value a separate pass over W gives), so a step after the first reads W
 * once less.  Errors: as uw_rk3_step. */
uw_status uw_rk3_steps(uw_mesh* mesh, const uw_physics* physics, double* W, double cfl,
                       double dt_fixed, double t_end, int32_t n_steps, double* t_dev,
                       void* stream);

/* The CFL time step alone: dt_dev (device double) = cfl * min_i
 * 2|Omega_i| / sum_p |l_p| (|u_i.n_p| + c_i), from cell averages W. */
uw_status uw_cfl_dt(uw_mesh* mesh, const uw_physics* physics, const double* W, double cfl,
                    double* dt_dev, void* stream);

/* Many independent meshes advanced together.  Every RK stage is one
 * persistent reconstruction launch per cell type over the tiles of all
 * instances plus one flux launch; the steps of uw_batch_rk3_step are
 * captured once into a hipGraph and replayed.  Every mesh must be
 * precomputed with the same scheme and live on one device; the batch copies
 * their tables (the meshes may be destroyed afterwards).
 * Batch state: device FP64 [V][N_total], N_total = sum of the instances'
 * cells; instance k occupies cells [cell_offsets[k], cell_offsets[k+1]) in
 * its own internal order.  Prescribed states and moving fronts stay with
 * their instance (each instance's fronts see its own time t_dev[k]).
 * Errors: UW_ESTATE (a mesh not precomputed), UW_EINVAL (meshes on
 * different devices or with different schemes, more than 2^28 cells, more
 * than 2^24 - 4 prescribed states or 2^30 front faces in total). */
uw_status uw_batch_create(uw_mesh* const* meshes, int32_t n, const uw_physics* physics,
                          uw_batch** out);
/* cell_offsets: host [n+1]. */
uw_status uw_batch_offsets(const uw_batch* batch, int64_t* cell_offsets);
/* n_steps SSP-RK3 steps of every instance, each with its own time step:
 * cfl * (instance's CFL bound) if dt_fixed <= 0, else dt_fixed, both
 * clamped to t_end - t_k.  t_dev: device [n] times, advanced on the device.
 * The first call with a given (W, t_dev, n_steps, cfl, dt_fixed, t_end)
 * captures a graph; later calls replay it (enqueued on `stream`). */
uw_status uw_batch_rk3_step(uw_batch* batch, double* W, double cfl, double dt_fixed,
                            double t_end, int32_t n_steps, double* t_dev, void* stream);

/* Chooses the tile size (256 or 512 cells; 512 only for FP32 WENO on the
 * conserved variables) and the launch schedule (number of persistent blocks
 * of the reconstruction kernels of each cell type and of the flux kernel:
 * one block per tile, or 1, 2, 4 or 8 blocks per compute unit; or one
 * reconstruction launch for both cell types) by timing residual
 * evaluations on the mesh or batch (exactly one of them) and stores both
 * there.  `cache_path` (nullable): a text file of earlier
 * choices keyed by the workload's shape, read first and appended to. */
uw_status uw_autotune(uw_mesh* mesh, uw_batch* batch, const uw_physics* physics,
                      const char* cache_path, void* stream);

/* Reads (get, nullable, host [3]) and/or sets (set, nullable) the launch
 * schedule of a mesh or batch (exactly one): persistent blocks of the
 * quadrilateral reconstruction, of the triangle reconstruction and of the
 * flux kernel; 0 = one block per tile.  A triangle entry of -1 puts both
 * cell types in one reconstruction launch of the quadrilateral entry's
 * blocks (not for the FP32 linear scheme, whose two kernels differ in
 * occupancy: there it means separate launches of one block per tile).
 * Other negative entries: UW_EINVAL.  Set is applied before get. */
uw_status uw_schedule(uw_mesh* mesh, uw_batch* batch, int32_t* get, const int32_t* set);

/* Tile size of a mesh or batch (exactly one): cells per tile, i.e. threads
 * per reconstruction and flux block, and the unit of LDS staging.  set =
 * 256 or 512 changes it (0 leaves it): the staging lists are rebuilt on the
 * host, the device tables are dropped after the device has finished queued
 * work (uploaded again on first use) and captured steps are retired.  512
 * serves FP32 WENO on the conserved variables only; other evaluations
 * then return UW_EINVAL.  get (nullable, host) receives the current size.
 * Default 256.  Errors: UW_EINVAL (size not 256 or 512), UW_EDEVICE,
 * UW_ENOMEM. */
uw_status uw_tile_size(uw_mesh* mesh, uw_batch* batch, int32_t set, int32_t* get);

/* Launch timing (tracing): with enable = 1 every later reconstruction and
 * flux launch of this mesh is bracketed by HIP events on the caller's
 * stream.  ms[0], ms[1] (nullable, host) receive the summed milliseconds of
 * the reconstruction and flux launches recorded so far and count[0..1] their
 * numbers; the records are then cleared.  enable = 0 stops recording,
 * enable = -1 leaves the setting unchanged.  Synchronises on the recorded
 * events when ms or count is given. */
uw_status uw_profile(uw_mesh* mesh, int32_t enable, double* ms, int64_t* count);

/* Synchronises `stream` and reports the device error flag of the mesh or
 * batch (UW_ENONFINITE), clearing it. */
uw_status uw_check(uw_mesh* mesh, uw_batch* batch, void* stream);

/* Free a mesh or batch and everything it holds on the device, after the
 * device has finished the work queued on it.  NULL is ignored. */
void uw_mesh_destroy(uw_mesh* mesh);
void uw_batch_destroy(uw_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* UWENO_H */
