/*
 * amr_oracle.h -- C API of the plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke
 * entry point and the CPU-baseline leg of the benchmark may load this
 * library.  It shares no code with the HIP path.
 *
 * The oracle follows the paper's description of the Enzo-P/Cello timestep
 * (Bordner & Norman, "Computational Cosmology and Astrophysics on Adaptive
 * Meshes using Charm++"):
 *   - array-of-octrees mesh, one Block per octree node (Sec. II-B);
 *   - ghost-zone refresh of a given width for the named fields, with
 *     Restrict/Prolong across refinement jumps (Sec. II-B);
 *   - the "ppm" Method, a modified piecewise-parabolic Euler solver
 *     (Sec. II-C), here directionally split with a two-shock Riemann solver.
 * The paper gives no formulas; every arithmetic detail is a stated reading,
 * written out next to the code that applies it.
 */
#ifndef AMR_ORACLE_H
#define AMR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_GHOST 3
#define ORC_NFIELD 5     /* rho, m_x, m_y, m_z, E; dual energy adds rho e */
#define ORC_MAXLEV 8

enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1 };

typedef struct {
  int32_t root[3];        /* octrees (root blocks) per axis                 */
  int32_t block_cells;    /* N: cells per block edge, even, >= 8            */
  int32_t max_level;      /* deepest refinement level allowed               */
  int32_t bc[3];          /* per axis, both faces: ORC_BC_*                 */
  double gamma, cfl, rho_floor, p_floor;
  int32_t riemann_iters;  /* fixed number of two-shock Newton iterations    */
  int32_t n_refine;       /* static refinement list: (level,i,j,k) x n      */
  const int32_t* refine;
  /* Dual-energy formalism (Bryan et al. 1995): a sixth field rho e (internal
   * energy density) advected with the flow and given the -p div(v) work; the
   * pressure comes from E - ke where (E - ke) > eta1 E, else from rho e; after
   * each sweep's update rho e is reset to E - ke where (E - ke) > eta2 E. */
  int32_t dual_energy;    /* 0: five fields; 1: six fields                  */
  double eta1, eta2;
} orc_desc;

typedef struct orc_mesh orc_mesh;

/* Build the balanced array-of-octrees described by d.  Returns 0 or <0. */
int orc_create(const orc_desc* d, orc_mesh** out);
/* Build from an explicit leaf list (level,i,j,k) x n; must tile the domain
 * and satisfy 2:1 balance (checked). */
int orc_create_from_leaves(const orc_desc* d, int64_t n, const int32_t* keys,
                           orc_mesh** out);
void orc_destroy(orc_mesh* m);
const char* orc_last_error(void);

int64_t orc_nleaf(const orc_mesh* m);
int orc_num_threads(void); /* OpenMP threads the oracle's loops use */
void orc_leaf_keys(const orc_mesh* m, int32_t* out /* 4 x nleaf */);
/* Padded block storage: U[leaf][field][z][y][x], edge M = N + 6; 5 fields,
 * or 6 with the dual-energy field (orc_nfields). */
int orc_nfields(const orc_mesh* m);
double* orc_state(orc_mesh* m);
int64_t orc_floor_count(const orc_mesh* m);

void orc_refresh(orc_mesh* m);
double orc_cfl_dt(const orc_mesh* m);
/* One full step: dt from CFL, refresh, three sweeps (xyz on even step
 * index, zyx on odd), reflux.  Returns dt. */
double orc_step(orc_mesh* m, int64_t step_index);
/* Same with a given dt (no CFL reduction). */
void orc_step_dt(orc_mesh* m, int64_t step_index, double dt);
/* Comoving coordinates (expansion factor a, H = adot / a at the step's mid
 * time): CFL dt = (C_cfl * a) * min dx / (|v| + c); the step runs the plain
 * step with dt / a, then the Crank-Nicolson expansion sources over dt. */
double orc_cfl_dt_comoving(const orc_mesh* m, double a);
void orc_step_comoving(orc_mesh* m, int64_t step_index, double dt, double a, double hubble);

/* Tracer particles.  Positions in level-0 cell units: X in [0, root[0]*N)
 * etc.; a particle belongs to the leaf holding level-l cell floor(X * 2^l).
 * orc_locate: that leaf, or -1 outside the domain.  orc_tracers_drift: one
 * drift of the alive particles with the velocity of the current state (its
 * ghosts must be refreshed) by trilinear interpolation of u = m / rho between
 * cell centres, X += (dt * u) * root[0] * N, periodic wrap; particles leaving
 * through an outflow face get alive = 0.  Returns how many were removed.
 * orc_step_tracers: dt from CFL, refresh, drift, then the hydro step. */
int64_t orc_locate(const orc_mesh* m, const double P[3]);
int64_t orc_tracers_drift(const orc_mesh* m, double dt, int64_t n, double* X, double* Y, double* Z,
                          int32_t* alive);
double orc_step_tracers(orc_mesh* m, int64_t step_index, int64_t n, double* X, double* Y, double* Z,
                        int32_t* alive);

/* Self-gravity step on a uniform periodic mesh (all leaves at level 0):
 * kick-drift-kick with g = -grad(phi), lap(phi) = 4 pi G (rho - mean rho) by
 * mg0 (ncycles V(nu1, nu2) cycles warm-started from phi, a global
 * (root[0] N) x (root[1] N) x (root[2] N) grid, x fastest); phi_current = 1
 * says phi already belongs to the current density (the previous step's
 * output), 0 solves it first.  On return phi belongs to the new density.
 * Returns dt, or -1 for a refined or non-periodic mesh. */
double orc_step_gravity(orc_mesh* m, int64_t step_index, double four_pi_G, double* phi, int phi_current,
                        int ncycles, int nu1, int nu2);

/* Comoving self-gravity step with the caller's dt, a at the step's start,
 * middle and end, H at its middle: half kick (dt/2) / a0^2 with phi of
 * lap(phi) = four_pi_G (rho - mean rho), the comoving hydro step, phi of the
 * new density, half kick (dt/2) / a1^2.  Returns 0, or -1 for a refined or
 * non-periodic mesh. */
int orc_step_gravity_comoving(orc_mesh* m, int64_t step_index, double dt, double a0, double a_mid, double a1,
                              double hubble, double four_pi_G, double* phi, int phi_current, int ncycles, int nu1,
                              int nu2);

/* Caller-driven branch tape (frozen-branch runs of any sequence of oracle
 * calls on this thread): record, then replay the recorded choices; stop
 * returns -1 if a replay did not consume them exactly, else 0. */
void orc_tape_record(void);
void orc_tape_replay(void);
int orc_tape_stop(void);

/* Frozen-branch central differences of the density misfit (reading R17 of
 * the adjoint: dt sequence and every discrete choice held at the base
 * run's).  From m's state (unchanged), nsteps steps of indices first_step,
 * first_step + 1, ... with the given dts; L = sum over active leaf cells of
 * 8^-level (rho - target)^2 (target: nleaf x N^3, x fastest).  The base
 * run records its choices; for each of the nidx flat density indices
 * (leaf * N^3 + (z N + y) N + x) the runs with rho +- eps replay them, and
 * grad_out[q] = (L(+eps) - L(-eps)) / (2 eps).  loss_out (may be NULL)
 * receives the base run's L.  Returns 0, or -1 (five fields only; a replay
 * that does not consume the recorded choices exactly). */
int orc_frozen_fd_density_grad(const orc_mesh* m, int64_t first_step, int nsteps, const double* dts,
                               const double* target, double eps, const int64_t* idx, int64_t nidx,
                               double* grad_out, double* loss_out);

/* Test hooks on the building blocks. */
#define ORC_DEBUG_SKIP_REFLUX 1
#define ORC_DEBUG_DE_PDV_SIGN 2   /* rho e takes +p div(v) */
#define ORC_DEBUG_DE_ENTHALPY 4   /* rho e flux with gamma / (gamma - 1) */
#define ORC_DEBUG_DE_ETA1_FLIP 8  /* pressure source selection reversed */
#define ORC_DEBUG_GRAVITY_SIGN 16 /* g = +grad(phi) */
#define ORC_DEBUG_GRAVITY_NO_A 32 /* comoving kicks without the 1/a^2 */
#define ORC_DEBUG_FLOOR_E_NO_KE 64     /* pressure floor resets E to p_floor/(gamma-1) alone */
#define ORC_DEBUG_FLOOR_KEEP_VEL 128   /* density floor keeps the velocity (momenta rescaled) */
#define ORC_DEBUG_DE_FLOOR_NO_IG 256   /* rho e floor set to p_floor, not p_floor/(gamma-1) */
#define ORC_DEBUG_EDGE_NO_FLOOR 512    /* traced edge states left unfloored */
#define ORC_DEBUG_CFL_SUM 1024         /* CFL signal speed |u|+|v|+|w|+c instead of max_d |u_d|+c */
#define ORC_DEBUG_EXP_FLOOR_NO_IG 2048 /* expansion raises E - ke to p_floor, not p_floor/(gamma-1) */
#define ORC_DEBUG_FLOOR_NO_COUNT 4096  /* density floor resets not counted */
void orc_set_debug(int flags);
void orc_riemann(const double* gas /* gamma,p_floor */, int iters,
                 const double* WL /* rho,u,v,w,p */, const double* WR,
                 double* state_out /* rho,u,v,w,p Godunov */, double* flux_out,
                 double* pstar_out, double* ustar_out);
/* Fluxes of one pencil of n conserved cells (rho, m_normal, m_t1, m_t2, E),
 * interfaces j+1/2 for j = 2 .. n-4; flux_out is 5 x (n-5). */
void orc_pencil_flux(const double* gas /* gamma,rho_floor,p_floor */, int iters,
                     double nu, int n, const double* U /* 5 x n */, double* flux_out);

/* mg0 Poisson solver (mg_oracle.c): the 7-point Laplacian of phi equals f
 * on a uniform periodic nx x ny x nz grid of spacing h (arrays x fastest).
 * f is made mean-free; ncycles V(nu1, nu2) cycles of red-black Gauss-Seidel
 * with residual restriction (8-child mean) and trilinear prolongation,
 * starting from phi; phi is returned with zero mean; resid (ncycles + 1
 * values, may be NULL) receives the residual L2 norm before and after each
 * cycle.  Returns the number of levels, or -1 for odd or too small sizes. */
#define ORC_MG_DEBUG_INJECT 1        /* piecewise-constant prolongation */
#define ORC_MG_DEBUG_RESTRICT_SUM 2  /* restriction sums instead of averaging */
#define ORC_MG_DEBUG_SMOOTH_SIGN 4   /* smoother adds h^2 f */
void orc_mg_set_debug(int flags);
int orc_mg_levels(int nx, int ny, int nz);
/* Building blocks: fine (2nxc x 2nyc x 2nzc) += prolongation of coarse;
 * coarse_f = restriction of the residual f - lap(phi) of a grid. */
void orc_mg_prolong_add(int nxc, int nyc, int nzc, const double* coarse, double* fine);
void orc_mg_restrict_residual(int nx, int ny, int nz, double h, const double* f, const double* phi,
                              double* coarse_f);
int orc_mg_solve(int nx, int ny, int nz, double h, const double* f, double* phi, int ncycles, int nu1, int nu2,
                 double* resid);

int orc_mg_vcycle_from_zero(int nx, int ny, int nz, double h, const double* f, double* phi, int nu1, int nu2);

/* mg0 on the octree (Sec. II-C gravity solver on the Sec. II-B array of
 * octrees): the composite-grid Poisson problem on the leaves of a periodic
 * 2:1-balanced mesh and its multigrid V-cycle; readings in amr_oracle.c.
 * Arrays are per leaf N^3 doubles (x fastest), leaves in m's order.
 * orc_mgc_apply: L phi.  orc_mgc_solve: f made mean-free (volume-weighted),
 * ncycles composite V(nu1, nu2) cycles from phi, phi returned with zero
 * volume-weighted mean, resid (ncycles + 1, may be NULL) the volume-weighted
 * residual L2 norms; an unrefined mesh takes orc_mg_solve's path exactly.
 * Return 0 (apply) or the number of levels (solve), -1 for a non-periodic
 * mesh or a coarsest level above 4096 cells. */
#define ORC_MGC_DEBUG_NO_MATCH 1  /* coarse side of a coarse-fine face keeps its own flux */
#define ORC_MGC_DEBUG_FLAT 2      /* coarse-fine ghosts without slopes (constant) */
void orc_mgc_set_debug(int flags);
int orc_mgc_apply(const orc_mesh* m, const double* phi, double* out);
int orc_mgc_solve(const orc_mesh* m, const double* f, double* phi, int ncycles, int nu1, int nu2, double* resid);

/* Self-gravity step on any periodic mesh (mg0 on the octree): phi on the
 * leaves (per leaf N^3, m's leaf order), otherwise as orc_step_gravity,
 * which it equals bit for bit on an unrefined mesh.  Returns dt, or -1. */
double orc_step_gravity_amr(orc_mesh* m, int64_t step_index, double four_pi_G, double* phi, int phi_current,
                            int ncycles, int nu1, int nu2);

/* Remesh (density-slope criterion).  Evaluates the per-leaf indicator on
 * refreshed data, applies refine/coarsen with 2:1 balance and the capacity
 * policy, and returns a new mesh holding the migrated state.  Counters:
 * out_stats[0]=refined, [1]=coarsened octets, [2]=refused refinements. */
int orc_remesh(orc_mesh* m, double refine_slope, double coarsen_slope,
               int64_t max_blocks, orc_mesh** out, int64_t* out_stats);
/* Per-leaf indicator S_b (max over active cells and axes of
 * |rho(+1)-rho(-1)| / (2 rho)).  Requires refreshed ghosts. */
void orc_indicator(const orc_mesh* m, double* out /* nleaf */);

#ifdef __cplusplus
}
#endif
#endif
