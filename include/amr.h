/*
 * amr.h -- C ABI of the MI355X (gfx950) AMR hydro hot path.
 *
 * One timestep over every leaf block of an array-of-octrees mesh, as the
 * paper describes the Enzo-P/Cello step (Bordner & Norman, "Computational
 * Cosmology and Astrophysics on Adaptive Meshes using Charm++"):
 *   - Sec. II-B: the mesh is an array of octrees, one Block per node; a
 *     Method acting on a Block needs a ghost layer of a stated width for the
 *     stated fields, refreshed from neighbouring Blocks, with Restrict and
 *     Prolong across refinement jumps; Boundary supplies physical ghosts;
 *     Refine decides where blocks split or merge;
 *   - Sec. II-C: the hydro Method is a modified piecewise-parabolic method.
 * Here the refresh, the CFL reduction, the three directionally split PPM
 * sweeps and the coarse-fine reflux run as HIP kernels on one GPU.
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev are device pointers (HIP global memory) that the
 *     caller allocates, owns and keeps alive until the stream work that uses
 *     them has finished.  The library never allocates device memory; it keeps
 *     no device pointer beyond a call, except the workspace given to
 *     amr_mesh_upload, which must stay allocated while the mesh is used.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Work is enqueued asynchronously on it unless stated otherwise.
 *   - Every call returns an amr_status; on failure amr_last_error() gives a
 *     message (per thread, valid until the next failing call).
 *   - Field storage U_dev: n_leaves blocks in the order of amr_mesh_blocks,
 *     each block = 5 fields (rho, m_x, m_y, m_z, E), 6 with the dual-energy
 *     field rho e (amr_mesh_desc.dual_energy), of M^3 FP64 values,
 *     M = N + 6 (ghost width 3 on each side), index (field, z, y, x) with x
 *     fastest, no padding: block stride n_fields M^3 doubles, field stride
 *     M^3.
 *     Only active cells (ghost-free interior N^3) carry state between calls;
 *     ghosts are scratch that a refresh overwrites.
 */
#ifndef AMR_H
#define AMR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amr_mesh amr_mesh;
/* A batch of independent meshes is a mesh handle whose leaves form one flat
 * worklist of several instances (amr_batch_create); every entry point that
 * takes an amr_mesh* also takes a batch. */
typedef struct amr_mesh amr_batch;
typedef struct amr_graph amr_graph;

typedef int32_t amr_status;
#define AMR_OK 0
#define AMR_E_INVALID (-1)  /* bad argument or descriptor */
#define AMR_E_BALANCE (-2)  /* leaf set violates the 2:1 rule or does not tile */
#define AMR_E_NOMEM (-3)    /* host allocation failed */
#define AMR_E_HIP (-4)      /* a HIP call or kernel launch failed */
#define AMR_E_CAPACITY (-5) /* remesh would exceed max_blocks */
#define AMR_E_STATE (-6)    /* call out of order (e.g. no workspace uploaded) */

#define AMR_BC_PERIODIC 0
#define AMR_BC_OUTFLOW 1 /* single-level meshes only */

/* Mesh description (Sec. II-B: array of octrees, Blocks of N^3 cells, ghost
 * width and fields named by the application).  Cells are cubic:
 * dx_l = 1 / (root[0] * N * 2^l); the domain is [0,1] x [0, root[1]/root[0]]
 * x [0, root[2]/root[0]]. */
typedef struct {
  int32_t root[3];        /* octrees per axis, >= 1                         */
  int32_t block_cells;    /* N: 8, 16 or 32                                 */
  int32_t ghost;          /* ghost width; must be 3                         */
  int32_t max_level;      /* deepest level, 0..7                            */
  int32_t bc[3];          /* AMR_BC_* per axis (both faces)                 */
  double gamma;           /* ratio of specific heats, > 1                   */
  double cfl;             /* Courant number of the dt reduction             */
  double rho_floor, p_floor; /* density and pressure floors, >= 1e-100; states
                             are expected within [floor, 1e100]       */
  int32_t riemann_iters;  /* fixed two-shock Newton iterations (e.g. 5)     */
  int32_t n_refine;       /* static refinement list, borrowed for the call: */
  const int32_t* refine;  /* n_refine x (level, i, j, k) block keys         */
  /* Dual-energy formalism (Bryan et al. 1995, the PPM variant the paper's
   * Sec. II-C Method derives from, for flows whose kinetic energy dwarfs the
   * thermal one): 1 adds a sixth field rho e (internal energy density) to
   * every cell.  A cell's pressure is (gamma-1)(E - ke) where E - ke > eta1 E,
   * else (gamma-1) rho e; rho e is carried by the internal-energy flux of the
   * Godunov state u_g p_g / (gamma-1) and takes the work -p div(v) (the cell
   * pressure times the difference of the Godunov velocities); after each
   * sweep's update rho e = E - ke where E - ke > eta2 E, then rho e is
   * floored at p_floor / (gamma-1) (counted).  The refresh, reflux, remesh
   * and comoving expansion treat rho e like the other fields; the adjoint
   * entries reject such meshes.  All instances of a batch must agree. */
  int32_t dual_energy;    /* 0 or 1                                         */
  double eta1, eta2;      /* in [0, 1]; typically 1e-3 and 0.1              */
} amr_mesh_desc;

typedef struct {
  int64_t n_leaves;
  int32_t block_cells;     /* N */
  int32_t padded;          /* M = N + 6 */
  int64_t block_stride;    /* doubles per block = n_fields M^3 */
  int64_t field_stride;    /* doubles per field = M^3 */
  int64_t field_bytes;     /* bytes of U_dev = n_leaves * block_stride * 8 */
  int64_t workspace_bytes; /* bytes the caller allocates for amr_mesh_upload */
  int64_t n_cf_faces;      /* coarse-fine block faces (both sides counted) */
  int32_t levels[8];       /* leaves per level */
  int64_t n_instances;     /* meshes in the handle (1 unless batched) */
  int64_t adjoint_scratch_bytes; /* scratch of amr_hydro_step_adjoint */
  int64_t adjoint_face_bytes;    /* scratch of amr_hydro_step_adjoint_recorded */
  int32_t n_fields;        /* 5 (rho, m_x, m_y, m_z, E), or 6 with rho e */
  int32_t pad0;
} amr_mesh_info_t;

/* Build the balanced array-of-octrees: roots, then each refine entry in
 * order (refining a leaf ancestor first when needed), then refinement until
 * no leaf touches (face, edge or corner, periodic wrap included) a leaf two
 * or more levels finer.  Sec. II-B (array-of-octrees, Refine).
 * Errors: AMR_E_INVALID for a bad descriptor (ghost != 3, N not in {8,16,32},
 * key out of range, outflow on a refined mesh), or more leaves than one
 * kernel launch over the leaves can cover (2^32 work items: 1,525,201 leaves
 * of 8^3, 381,300 of 16^3, 69,615 of 32^3; also for the meshes of
 * amr_mesh_create_from_leaves, amr_batch_create and a remesh). */
amr_status amr_mesh_create(const amr_mesh_desc* desc, amr_mesh** out);

/* Build from an explicit leaf set (n x (level,i,j,k), borrowed for the
 * call): the octree of Sec. II-B given by its leaves (checkpoint restart,
 * meshes made elsewhere).  Errors: AMR_E_BALANCE if the leaves do not tile
 * the domain or violate the 2:1 rule. */
amr_status amr_mesh_create_from_leaves(const amr_mesh_desc* desc, int64_t n,
                                       const int32_t* keys, amr_mesh** out);

/* Batched meshes: n independent meshes (each its own array of octrees, gas,
 * boundaries and static refinement; all with the same block_cells) in one
 * handle whose leaves form one flat worklist: instance 0's leaves first,
 * each instance's in its own storage order.  Every step entry point then
 * advances all instances in the same launches, each with its own dt:
 * dt_dev holds n doubles.  This is the paper's "agglomerating work units"
 * (Sec. IV) applied to many small meshes on one GPU.  Remesh is for
 * single meshes. */
amr_status amr_batch_create(const amr_mesh_desc* descs, int32_t n, amr_batch** out);
/* One step of every instance of a batch (Sec. II-C ppm Method on every
 * Block of every instance, Sec. IV agglomerated work units): amr_hydro_step
 * on the batch handle -- each instance's refresh, its own CFL dt (dt_dev:
 * n_instances doubles, written), sweeps and reflux, all instances in the same
 * launches.  Errors as amr_hydro_step. */
amr_status amr_batch_step(amr_batch* batch, double* U_dev, double* dt_dev, int64_t step_index, void* stream);
/* first_leaf[m] = index of instance m's first leaf, first_leaf[n] =
 * n_leaves (host memory, cap >= n_instances + 1).  Not in the paper (the
 * batch's leaf layout, reading of Sec. IV's agglomeration). */
amr_status amr_mesh_instance_offsets(const amr_mesh* mesh, int64_t* first_leaf, int64_t cap);

/* Release the host tables of a mesh or batch (Sec. II-B: the mesh object;
 * the device memory is the caller's). */
amr_status amr_mesh_destroy(amr_mesh* mesh);
/* Sizes of the storage the caller allocates for a mesh: leaves per level,
 * field layout, workspace and scratch bytes (Sec. II-B: Data of the Blocks,
 * Field layout). */
amr_status amr_mesh_info(const amr_mesh* mesh, amr_mesh_info_t* out);

/* Leaf keys (level, i, j, k) in storage order (roots x-fastest, Morton order
 * inside each octree; Sec. II-B array of octrees, one Block per node), for
 * initial conditions (Sec. II-B Initial).  keys_out holds cap x 4 int32
 * (host memory). */
amr_status amr_mesh_blocks(const amr_mesh* mesh, int32_t* keys_out, int64_t cap);

/* Copy the mesh tables into caller-owned device memory of workspace_bytes
 * (amr_mesh_info) and bind it to the mesh.  The copy is enqueued on the
 * stream; the workspace must outlive every later call on this mesh.  Not in
 * the paper (the device copy of the Sec. II-B neighbour and refresh
 * relations). */
amr_status amr_mesh_upload(amr_mesh* mesh, void* workspace_dev, void* stream);

/* Ghost refresh (Sec. II-B): fill the width-3 ghost shell of all fields of
 * every leaf.  Phase 1: same-level copies (faces, edges, corners; periodic
 * wrap; outflow = nearest domain cell), restriction (mean of the 8 children)
 * into ghosts covered by finer leaves.  Phase 2: minmod-limited linear
 * prolongation into ghosts covered by a coarser leaf. */
amr_status amr_refresh_ghosts(amr_mesh* mesh, double* U_dev, void* stream);

/* CFL dt (device, 1 double per instance): C_cfl * min over active leaf
 * cells of dx_l / (max_d |u_d| + c).  Exact minimum, order independent.
 * Not in the paper (reading: one global dt per mesh, the step's stability
 * limit for the Sec. II-C ppm Method). */
amr_status amr_cfl_dt(amr_mesh* mesh, const double* U_dev, double* dt_dev, void* stream);

/* One hydro step (Sec. II-C "ppm" Method on every Block, after the refresh
 * its ghosts need): dt from the CFL reduction written to dt_dev, refresh,
 * PPM sweeps x,y,z on even step_index and z,y,x on odd, then reflux at
 * coarse-fine faces.  U_dev is updated in place. */
amr_status amr_hydro_step(amr_mesh* mesh, double* U_dev, double* dt_dev, int64_t step_index,
                          void* stream);

/* Comoving coordinates (Sec. II-C: the ppm Method with cosmological
 * comoving expansion terms; the terms of Bryan et al. 1995).  x is the
 * comoving position, v the peculiar velocity, a the expansion factor and
 * H = adot / a.  amr_cfl_dt_comoving: dt = (C_cfl * a) * min over active
 * leaf cells of dx_l / (max_d |v_d| + c) (a > 0, finite).
 * amr_hydro_step_comoving: with dt given on the device (e.g. from the CFL
 * call) and a, H taken at the step's mid time, runs the plain step with
 * dt / a (the flux divergence carries 1/a; the per-instance dt / a is kept in
 * the workspace), then the expansion sources on every active cell with
 * Crank-Nicolson factors, c = (dt / 2) H: momenta times (1 - c) / (1 + c),
 * internal energy times (1 - 3 (gamma - 1) c) / (1 + 3 (gamma - 1) c), the
 * total energy updated by both changes (H = 0 leaves the state bit for bit;
 * where the source lowers the internal energy below the pressure floor it is
 * raised to it and counted in amr_floor_count).  Stream-ordered; U_dev is
 * updated in place; AMR_E_INVALID for a <= 0 or non-finite a, H. */
amr_status amr_cfl_dt_comoving(amr_mesh* mesh, const double* U_dev, double a, double* dt_dev, void* stream);
amr_status amr_hydro_step_comoving(amr_mesh* mesh, double* U_dev, const double* dt_dev, int64_t step_index,
                                   double a, double hubble, void* stream);

/* A run of comoving steps with the expansion history evaluated on the
 * device (not in the paper: a flat matter + Lambda background,
 * H(a) = H0 sqrt(omega_m / a^3 + omega_l), omega_m + omega_l = 1, for which
 * a(t) has a closed form; radiation neglected).  cosmo_dev: 4 doubles on the
 * device, [0] the time t (in: at the first step; out: after the last),
 * [1] a(t) at the last step's start, [2] a and [3] H at its mid time.  Each
 * step: a(t); the comoving CFL dt into dt_dev[k] (nsteps doubles); a and H
 * at t + dt / 2; amr_hydro_step_comoving with them (step index
 * first_step + k); t += dt.  Nothing is read back to the host, so the run
 * can be captured in a graph.  Single meshes only (AMR_E_INVALID for a
 * batch); AMR_E_INVALID for H0 <= 0, omega_m <= 0, omega_l < 0 or
 * |omega_m + omega_l - 1| > 1e-12. */
amr_status amr_hydro_steps_comoving(amr_mesh* mesh, double* U_dev, double* dt_dev, int64_t nsteps,
                                    int64_t first_step, double H0, double omega_m, double omega_l,
                                    double* cosmo_dev, void* stream);

/* Adjoint of the comoving step (Sec. II-C comoving terms; the adjoint itself
 * is not in the paper: reading R17, every step's dt, a and H frozen at the
 * forward's values).  amr_hydro_step_comoving_record runs
 * amr_hydro_step_comoving (dt_dev given, a and H at the mid time) from U_dev
 * as amr_hydro_step_record does from a plain step: U_dev is refreshed in
 * place (it becomes S0), S1_dev and S2_dev receive the second and third
 * sweeps' inputs, U_pre_dev the state after the reflux and before the
 * expansion sources, U_out_dev the step's result, floors_dev the sweeps'
 * floor-reset count (the expansion's own resets are counted in
 * amr_floor_count only).  amr_hydro_step_comoving_adjoint_recorded: on entry
 * lam_dev holds dL/dU after the step (ghost entries zero), on exit dL/dU
 * before it: the transpose of the expansion sources at U_pre_dev (each
 * cell's floor decision held), then the plain step's transposes with dt / a
 * (floors_host as for amr_hydro_step_adjoint_recorded; scratch_dev:
 * adjoint_face_bytes of amr_mesh_info).  With the dual-energy field the
 * sixth field's adjoint takes the internal-energy factor (zero where its
 * floor was applied).
 * Errors: AMR_E_INVALID for a null or aliased buffer, a <= 0 or non-finite
 * a, H, floors_host < -1, riemann_iters > 8. */
amr_status amr_hydro_step_comoving_record(amr_mesh* mesh, double* U_dev, const double* dt_dev, double a,
                                          double hubble, double* S1_dev, double* S2_dev, double* U_pre_dev,
                                          double* U_out_dev, uint64_t* floors_dev, int64_t step_index,
                                          void* stream);
amr_status amr_hydro_step_comoving_adjoint_recorded(amr_mesh* mesh, const double* S0_dev, const double* S1_dev,
                                                    const double* S2_dev, const double* U_pre_dev,
                                                    const double* dt_dev, double a, double hubble,
                                                    const uint64_t* floors_dev, int64_t floors_host,
                                                    double* lam_dev, void* scratch_dev, int64_t step_index,
                                                    void* stream);

/* Sec. II-C ppm Method on every Block, repeated; the fused CFL is not in
 * the paper (reading: a step's dt needs only its predecessor's output).
 * nsteps consecutive hydro steps (step indices first_step, first_step + 1,
 * ...; U_dev updated in place): the same results as that many
 * amr_hydro_step calls, bit for bit, with step i's dt (one per instance) in
 * dt_dev[i * n_instances ...] (device, nsteps * n_instances doubles).  Only
 * the first step runs the CFL reduction over the state; each later step's dt
 * comes from its predecessor, whose last sweep adds the candidates of the
 * cells it updates and no reflux changes, and a kernel after the reflux
 * those of the refluxed cells (the minimum is exact in any order).  The
 * caller must not change U_dev between the steps of one call.
 * Stream-ordered; AMR_E_INVALID for nsteps < 0 or a null dt_dev. */
amr_status amr_hydro_steps(amr_mesh* mesh, double* U_dev, double* dt_dev, int64_t nsteps, int64_t first_step,
                           void* stream);
/* Sec. II-B refresh skipped where it would rewrite what is there (not in the
 * paper: the remesh of Sec. II-B Refine has just refreshed).
 * amr_hydro_steps for a state whose ghosts are current: the first step
 * skips its ghost refresh (the later ones refresh as usual).  The caller
 * guarantees that U_dev's ghost cells hold what a refresh would write, i.e.
 * that no active cell changed since the last amr_refresh_ghosts on this mesh
 * or since an amr_remesh_plan that refined and coarsened nothing (which
 * refreshes U_dev itself); then the results equal amr_hydro_steps bit for
 * bit.  For adaptive runs, whose remesh already refreshed the state. */
amr_status amr_hydro_steps_fresh(amr_mesh* mesh, double* U_dev, double* dt_dev, int64_t nsteps, int64_t first_step,
                                 void* stream);

/* The same step (Sec. II-C ppm Method after the Sec. II-B refresh) with dt
 * given on the device (no CFL reduction). */
amr_status amr_hydro_step_dt(amr_mesh* mesh, double* U_dev, const double* dt_dev,
                             int64_t step_index, void* stream);

/* Not in the paper (a launch-overhead reading of Sec. IV's agglomeration:
 * the fixed kernel sequence of two steps recorded once).
 * HIP graph of two consecutive steps (first_step and first_step+1, so one
 * even and one odd sweep order) bound to U_dev and dt_dev, captured on a
 * non-null stream; each launch advances the state by two steps.  The
 * second step's CFL reduction is fused into the first step, as in
 * amr_hydro_steps, and both steps use the ninst doubles at dt_dev (after a
 * launch they hold the second step's dt).  The captured kernels read and
 * write the same buffers every launch. */
amr_status amr_graph_create(amr_mesh* mesh, double* U_dev, double* dt_dev, int64_t first_step, void* stream,
                            amr_graph** out);
/* Replay the two captured steps on the stream. */
amr_status amr_graph_launch(amr_graph* graph, void* stream);
/* Release the graph (its captured buffers stay the caller's). */
amr_status amr_graph_destroy(amr_graph* graph);

/* Differentiation is not in the paper (reading R17: the exact vector-
 * Jacobian product of the Sec. II-C ppm step and the Sec. II-B refresh with
 * every discrete choice frozen).
 * The recording step, amr_hydro_step_adjoint_recorded and
 * amr_refresh_ghosts_adjoint, and amr_hydro_step_adjoint (recomputing), also
 * take a mesh with the dual-energy field (six fields: the sixth field's
 * adjoint passes through the pressure selection, its flux, the work term and
 * the resynchronisation and floors of the update).
 *
 * One hydro step (as amr_hydro_step, bitwise the same result) that keeps
 * what its adjoint needs, for reverse-mode differentiation without
 * recomputation: U_dev's ghosts are refreshed in place and U_dev is otherwise
 * not modified (it becomes the first sweep's input S0); the first and second
 * sweeps write their results to S1_dev and S2_dev, the third sweep and the
 * reflux write the new state to U_out_dev (field_bytes each, all distinct;
 * ghost cells of U_out_dev are unspecified: the next step's refresh fills
 * them); floors_dev (one uint64 on the device) receives the number of
 * post-update floor resets of this step.  dt_dev receives the CFL dt. */
amr_status amr_hydro_step_record(amr_mesh* mesh, double* U_dev, double* dt_dev, double* S1_dev, double* S2_dev,
                                 double* U_out_dev, uint64_t* floors_dev, int64_t step_index, void* stream);

/* Adjoint of one hydro step with its dt frozen (Sec. II-C Method, the
 * refresh of Sec. II-B): on entry lam_dev holds dL/dU after the step (ghost
 * entries zero), on exit dL/dU before it (ghost entries zero).  U_in_dev is
 * the state the forward step started from (a checkpoint), dt_dev the dt it
 * used, step_index its index (sweep order).  The step's sweep inputs are
 * recomputed into scratch_dev (adjoint_scratch_bytes of amr_mesh_info; the
 * mesh's floor-reset count is left unchanged); every limiter, flattening,
 * wave-direction, floor and Riemann branch is taken as the forward took it,
 * and the result is the exact vector-Jacobian product of the computed step
 * on those branches (post-update floors included).  The refresh transpose
 * scatter-adds with FP64 atomics (sums in unspecified order).
 * Errors: AMR_E_INVALID if riemann_iters exceeds 8. */
amr_status amr_hydro_step_adjoint(amr_mesh* mesh, const double* U_in_dev, const double* dt_dev, double* lam_dev,
                                  void* scratch_dev, int64_t step_index, void* stream);

/* The same adjoint from what amr_hydro_step_record kept: S0_dev (its U_dev
 * after the call), S1_dev, S2_dev, dt_dev and floors_dev (zero resets lets
 * the sweeps' transposes skip the floors).  floors_host: the value of
 * *floors_dev if the caller has read it (then only the matching transpose
 * kernels are launched; a value that differs from *floors_dev gives a wrong
 * result), or -1 (the kernels read the count on the device).  scratch_dev:
 * adjoint_face_bytes of amr_mesh_info.  Nothing is recomputed.
 * Errors: AMR_E_INVALID for floors_host < -1. */
amr_status amr_hydro_step_adjoint_recorded(amr_mesh* mesh, const double* S0_dev, const double* S1_dev,
                                           const double* S2_dev, const double* dt_dev, const uint64_t* floors_dev,
                                           int64_t floors_host, double* lam_dev, void* scratch_dev,
                                           int64_t step_index, void* stream);

/* Transpose of amr_refresh_ghosts at the refreshed state U_ref_dev (its
 * minmod slope choices): on entry lam_dev holds an adjoint on every cell,
 * ghosts included; on exit the ghost entries are folded into their source
 * cells and cleared. */
amr_status amr_refresh_ghosts_adjoint(amr_mesh* mesh, const double* U_ref_dev, double* lam_dev, void* stream);

/* Tracer particles (Sec. II-B: particles live on Blocks, are allocated in
 * fixed-size batches and move between Blocks; Sec. III: the blast workload
 * carries tracers).  Positions are in level-0 cell units: X in
 * [0, root[0] N), Y in [0, root[1] N), Z in [0, root[2] N); a particle belongs
 * to the leaf holding its level-l cell floor(X 2^l).  A set stores
 * `capacity` slots per leaf (a multiple of the 256-slot batch; n_leaves x
 * capacity below 2^32, the slots one kernel launch covers, else the calls
 * return AMR_E_INVALID), device memory owned by the caller:
 *   pos   3 x n_leaves x capacity doubles: every slot's X, then Y, then Z
 *         (slot s of leaf b at b * capacity + s);
 *   id    n_leaves x capacity int64, carried along;
 *   count n_leaves int32: leaf b holds slots 0 .. count[b]-1. */
typedef struct {
  double* pos;
  int64_t* id;
  int32_t* count;
} amr_tracer_set_t;
/* Bytes of the scratch the tracer calls need for this capacity; the scratch
 * must be zero-filled before its first use and is then kept by the caller
 * from call to call. */
amr_status amr_tracer_scratch_bytes(const amr_mesh* mesh, int64_t capacity, int64_t* bytes);
/* Advance every particle of `in` by one step into `out` (a distinct set):
 * drift with the velocity of U_dev (ghosts refreshed) -- per cell
 * u = m (1/rho), trilinear between the 8 cell centres around the particle --
 * X += (dt u) (root[0] N) with the instance's dt_dev entry; periodic axes wrap,
 * particles leaving through an outflow face are removed; then each particle
 * is written to the leaf holding its new position: those that stay keep
 * their order, arrivals are appended in no particular order.  The input
 * positions are overwritten.  Particles beyond a leaf's capacity are dropped
 * and counted (amr_tracer_counters). */
amr_status amr_tracers_advance(amr_mesh* mesh, const double* U_dev, const double* dt_dev,
                               const amr_tracer_set_t* in, amr_tracer_set_t* out, int64_t capacity,
                               void* scratch_dev, void* stream);
/* A hydro step (as amr_hydro_step) that advances the tracers of `in` into
 * `out` between the ghost refresh and the sweeps. */
amr_status amr_hydro_step_tracers(amr_mesh* mesh, double* U_dev, double* dt_dev, const amr_tracer_set_t* in,
                                  amr_tracer_set_t* out, int64_t capacity, void* scratch_dev, int64_t step_index,
                                  void* stream);
/* After a remesh: move every particle of old_set (the set of the mesh given
 * to amr_remesh_plan, old_leaves leaves) into new_set on new_mesh (made by
 * amr_remesh_plan and uploaded): particles of a kept leaf stay with it, those
 * of a split leaf go to the child holding their position, those of merged
 * leaves to the new parent; the order inside a leaf is not specified.
 * Positions are unchanged.  scratch_dev: the scratch of new_mesh for this
 * capacity (zero-filled before its first use). */
amr_status amr_tracers_remesh(amr_mesh* new_mesh, int64_t old_leaves, const amr_tracer_set_t* old_set,
                              amr_tracer_set_t* new_set, int64_t capacity, void* scratch_dev, void* stream);
/* Cumulative counters of the scratch (synchronises the stream): out3[0]
 * particles dropped for lack of capacity, [1] removed through outflow faces,
 * [2] lost (moved more than a leaf in one step: never under a CFL number
 * below 1).  reset != 0 zeroes them afterwards. */
amr_status amr_tracer_counters(amr_mesh* mesh, void* scratch_dev, int64_t capacity, int64_t* out3, int32_t reset,
                               void* stream);

/* Number of post-update floor resets since upload (synchronises the
 * stream).  Not in the paper (the positivity floors of the ppm reading). */
amr_status amr_floor_count(amr_mesh* mesh, int64_t* out, void* stream);

/* Remesh (Sec. II-B "Refine"; the paper's blast test refines adaptively).
 * Indicator per leaf: S_b = max over active cells and axes of
 * |rho(+1) - rho(-1)| / (2 rho) on refreshed data.  Rule: leaves with
 * S_b > refine_slope below max_level are refined in (S_b descending, then
 * level, z, y, x) order, each with the minimal refinement that keeps 2:1
 * balance, accepted only if that refines pre-existing leaves only (one level
 * per remesh) and the leaf count stays <= max_blocks (refused otherwise; the
 * library also refuses growth beyond the leaves one kernel launch can cover,
 * as amr_mesh_create states);
 * then, finer first, octets of pre-existing leaves all below coarsen_slope
 * merge if balance allows.  Data: kept leaves copy, new children prolong
 * (the refresh prolongation), merged parents restrict. */
typedef struct {
  double refine_slope, coarsen_slope;
  int64_t max_blocks;
} amr_remesh_params;
typedef struct {
  int64_t refined;    /* nodes split (including balance refinements) */
  int64_t coarsened;  /* octets merged */
  int64_t refused;    /* refinement candidates refused */
  int64_t n_leaves;   /* leaves of the new mesh */
} amr_remesh_stats;

/* Refreshes U_dev's ghosts, evaluates the indicator on the GPU, copies it to
 * the host (synchronises the stream) and builds the new mesh (host-owned,
 * destroy with amr_mesh_destroy).  U_dev must not change before
 * amr_remesh_apply.  When nothing is refined or coarsened (every candidate
 * refused, or none), *new_mesh_out is NULL: the mesh and U_dev stay as they
 * are (U_dev's ghosts now refreshed, see amr_hydro_steps_fresh), and stats
 * still count the refusals. */
amr_status amr_remesh_plan(amr_mesh* mesh, double* U_dev, const amr_remesh_params* params,
                           amr_mesh** new_mesh_out, amr_remesh_stats* stats, void* stream);
/* The same decisions from a caller-supplied indicator (S_host: n_leaves
 * doubles in host memory, storage order); no GPU work.  The returned mesh
 * (NULL when nothing changed) can be uploaded and migrated with
 * amr_remesh_apply like the one above. */
amr_status amr_remesh_plan_host(amr_mesh* mesh, const double* S_host, const amr_remesh_params* params,
                                amr_mesh** new_mesh_out, amr_remesh_stats* stats);
/* Fill the active cells of U_new_dev (new mesh layout) from U_old_dev (the
 * state given to amr_remesh_plan).  new_mesh must have been uploaded. */
amr_status amr_remesh_apply(amr_mesh* new_mesh, const double* U_old_dev, double* U_new_dev, void* stream);
/* The indicator alone into ind_dev (n_leaves doubles, device); ghosts of U_dev
 * must be refreshed. */
amr_status amr_indicator(amr_mesh* mesh, const double* U_dev, double* ind_dev, void* stream);

/* Launch shapes (not in the paper: Sec. IV's multiple kernel versions, one
 * per hardware choice).  Every choice computes bitwise-identical results
 * (each cell's arithmetic is the same; only the thread mapping changes). */
typedef struct {
  int32_t sweep_mode[3];  /* per axis x,y,z: 0 = one lane walks one pencil with
                             a register window; 1 = LDS-staged tile of whole
                             pencils, one thread per cell */
  int32_t sweep_block;    /* workgroup size of mode 0 (64..1024, multiple of 64) */
  int32_t refresh_block;  /* workgroup size of the refresh kernels */
  int32_t reflux_block;   /* workgroup size of the reflux kernels */
} amr_launch_t;
amr_status amr_mesh_set_launch(amr_mesh* mesh, const amr_launch_t* cfg);
amr_status amr_mesh_get_launch(const amr_mesh* mesh, amr_launch_t* cfg);

/* Per-phase kernel timing with HIP events recorded on the launch stream
 * around every kernel of refresh, CFL, sweeps and reflux (not in the paper:
 * measurement).  Phases: */
#define AMR_PHASE_CFL 0
#define AMR_PHASE_REFRESH1 1
#define AMR_PHASE_REFRESH2 2
#define AMR_PHASE_SWEEP_X 3
#define AMR_PHASE_SWEEP_Y 4
#define AMR_PHASE_SWEEP_Z 5
#define AMR_PHASE_REFLUX 6
/* amr_hydro_step_adjoint: recompute of the sweep inputs (copies, refresh,
 * two sweeps), reflux transpose, sweep transposes, refresh transpose */
#define AMR_PHASE_ADJ_RECOMPUTE 7
#define AMR_PHASE_ADJ_REFLUX 8
#define AMR_PHASE_ADJ_SWEEP_X 9
#define AMR_PHASE_ADJ_SWEEP_Y 10
#define AMR_PHASE_ADJ_SWEEP_Z 11
#define AMR_PHASE_ADJ_REFRESH 12
/* tracer drift and migration (amr_hydro_step_tracers, amr_tracers_advance) */
#define AMR_PHASE_TRACERS 13
/* expansion sources of amr_hydro_step_comoving and amr_hydro_step_gravity_comoving */
#define AMR_PHASE_EXPANSION 14
/* amr_poisson_solve (one record per solve), and the gravity steps' solves and kicks */
#define AMR_PHASE_POISSON 15
#define AMR_NPHASE 16
/* mg0 Poisson solver: the gravity Method's geometric multigrid V-cycle
 * (Sec. II-C; the self-gravity solver of the uniform-mesh cosmology test of
 * Sec. III).  Solves the 7-point Laplacian (sum of the 6 neighbours -
 * 6 phi) / dx^2 = f on a uniform periodic mesh: one instance, every leaf at
 * level 0, periodic on every axis, grid (root[0] N) x (root[1] N) x
 * (root[2] N) of spacing dx = dx_0.  Levels: level l+1 halves every axis of
 * level l while all of level l's axes are multiples of 4; the coarsest level
 * must hold at most 4096 cells.  A V(nu1, nu2) cycle: nu1 red-black
 * Gauss-Seidel sweeps (red = (i + j + k) even first; phi = (S - dx^2 f) / 6,
 * S = ((W + E) + (S + N)) + (B + T)), the coarse right-hand side = mean of
 * the 8 children's residuals, the coarse correction from 0 (64 red-black
 * sweeps on the coarsest level), trilinear prolongation of the correction
 * (weights 27, 9, 3, 1 over 64), nu2 sweeps.
 *   f_dev, phi_dev: n_leaves x N^3 doubles on the device, per leaf its cells
 *     x fastest, leaves in the order of amr_mesh_blocks (f_dev is read only;
 *     they may be the same buffer).  f is made mean-free first (periodic
 *     solvability); phi_dev holds the initial guess on entry and, after
 *     ncycles cycles, the mean-free result.
 *   resid_dev: null, or ncycles + 1 doubles on the device that receive the
 *     residual L2 norm sqrt(sum r^2) before the first cycle and after each.
 *   work_dev: amr_poisson_workspace_bytes bytes of device memory (the level
 *     arrays and reduction scratch), owned by the caller, contents ignored.
 * Means and norms are fixed-order two-stage sums (results are reproducible
 * from run to run; they differ from a sequential sum in the last bits).
 * Errors: AMR_E_INVALID for a batch, a refined mesh, a non-periodic axis, a
 * coarsest level above 4096 cells, ncycles < 0 or nu outside [0, 64], null
 * pointers (resid_dev excepted); AMR_E_STATE before amr_mesh_upload. */
amr_status amr_poisson_workspace_bytes(const amr_mesh* mesh, int64_t* bytes);
amr_status amr_poisson_solve(amr_mesh* mesh, const double* f_dev, double* phi_dev, int32_t ncycles, int32_t nu1,
                             int32_t nu2, double* resid_dev, void* work_dev, void* stream);

/* amr_poisson_solve without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, fixed-memory serving
 * loops, harnesses that forbid allocation): the solver's level arrays and
 * reduction scratch live in a fixed 64 MiB device buffer of the library,
 * one per GPU, held until the process ends.  Grids whose workspace
 * (amr_poisson_workspace_bytes) exceeds 64 MiB are refused with
 * AMR_E_CAPACITY; 128^3 cells (38.4 MB) fit.  The call allocates nothing.
 * Every call on one GPU shares that GPU's buffer: calls that overlap on one
 * GPU (concurrent streams or threads) race and must be serialised by the
 * caller.  The buffer's contents are ignored on entry, as work_dev's are.
 * Arguments, results and other errors as amr_poisson_solve; its results are
 * bit for bit those of amr_poisson_solve. */
amr_status amr_poisson_solve_static(amr_mesh* mesh, const double* f_dev, double* phi_dev, int32_t ncycles,
                                    int32_t nu1, int32_t nu2, double* resid_dev, void* stream);

/* Self-gravity step on the same meshes as amr_poisson_solve (the gravity
 * Method coupled to ppm, Sec. II-C; the self-gravitating gas of Sec. III):
 * kick-drift-kick.  phi solves lap(phi) = four_pi_G (rho - mean rho) with
 * ncycles V(nu1, nu2) cycles warm-started from phi_dev; a half kick with
 * g = -grad(phi) (central differences (phi(a-1) - phi(a+1)) / (2 dx),
 * periodic) changes the momentum by (dt/2) rho g and the total energy by the
 * kinetic-energy change, so it changes no internal energy (nor the
 * dual-energy field); then the hydro step (as amr_hydro_step: dt_dev
 * receives the CFL dt), phi of the new density, the second half kick.
 *   phi_dev: n_leaves x N^3 doubles (the amr_poisson_solve layout), the
 *     mean-free potential; phi_current = 1 says it belongs to U's density
 *     (the previous call's output), 0 makes the call solve it first.  On
 *     return it belongs to the new density.
 *   work_dev: amr_poisson_workspace_bytes bytes.
 * four_pi_G = 0 (with phi_dev zero) gives amr_hydro_step bit for bit.
 * Errors: those of amr_poisson_solve, and of amr_hydro_step. */
amr_status amr_hydro_step_gravity(amr_mesh* mesh, double* U_dev, double* dt_dev, int64_t step_index,
                                  double four_pi_G, double* phi_dev, int32_t phi_current, int32_t ncycles,
                                  int32_t nu1, int32_t nu2, void* work_dev, void* stream);

/* Comoving self-gravity step (the gravity Method with the comoving ppm
 * Method, Sec. II-C; the comoving terms of Bryan et al. 1995), on the same
 * meshes as amr_poisson_solve.  phi is the comoving potential, free of a:
 * lap(phi) = four_pi_G (rho - mean rho) (the comoving density; four_pi_G
 * carries the cosmology, e.g. 3/2 Omega_m H0^2 for code units in which
 * mean rho = 1), and the peculiar acceleration is -grad(phi) / a^2 at the
 * time of each kick.  With dt given on the device (e.g. from
 * amr_cfl_dt_comoving) and a0, a_mid, a1 the expansion factors at the
 * step's start, middle and end, H = adot / a at the middle:
 *   half kick (dt/2) / a0^2 with phi of U's density (solved first unless
 *     phi_current);
 *   expansion sources over dt/2 (the Crank-Nicolson factors of
 *     amr_hydro_step_comoving with c = (dt/4) H);
 *   the plain refresh, sweeps and reflux with dt / a_mid;
 *   expansion sources over dt/2;
 *   phi of the new density, half kick (dt/2) / a1^2.
 * a0 = a_mid = a1 = 1, H = 0 gives amr_hydro_step_gravity with the same dt
 * bit for bit.  Layouts, phi_current and work_dev as amr_hydro_step_gravity;
 * dt_dev is read only.  Errors: those of amr_hydro_step_gravity, and
 * AMR_E_INVALID for an expansion factor <= 0 or not finite, or a non-finite
 * H or four_pi_G. */
amr_status amr_hydro_step_gravity_comoving(amr_mesh* mesh, double* U_dev, const double* dt_dev, int64_t step_index,
                                           double a0, double a_mid, double a1, double hubble, double four_pi_G,
                                           double* phi_dev, int32_t phi_current, int32_t ncycles, int32_t nu1,
                                           int32_t nu2, void* work_dev, void* stream);

/* on != 0 starts recording (clearing earlier records); 0 stops. */
amr_status amr_profile_enable(amr_mesh* mesh, int32_t on);
/* Waits for the recorded events, then writes per phase the summed kernel
 * milliseconds (ms_out) and the number of launches (launches_out), each of
 * AMR_NPHASE entries (host memory), and clears the records. */
amr_status amr_profile_read(amr_mesh* mesh, double* ms_out, int64_t* launches_out);

/* Not in the paper (a check of this build's arithmetic).
 * Device arithmetic self-test.  The kernels take reciprocals and square
 * roots of positive operands in [2^-767, 2^1022] (densities, pressures,
 * sound speeds, shock mass fluxes: within that range for floors >= 1e-100
 * and states <= 1e100) with the IEEE sequences minus their operand scaling
 * and special-value fix-ups, which are identities on that range.  This
 * call compares both with the IEEE 1/x and sqrt(x) on n operands (random
 * mantissas, exponents uniform over [-767, 1022], from seed) and adds the
 * numbers of differing reciprocals and square roots to counts[0] and
 * counts[1] (device memory, 2 x uint64, not cleared).  Stream-ordered. */
amr_status amr_arith_selftest(uint64_t seed, int64_t n, uint64_t* counts_dev, void* stream);

/* Message of the last failing call on this thread (not in the paper). */
const char* amr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
