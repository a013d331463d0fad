// kernels.hpp -- launchers of the gfx950 kernels of one hydro step.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.hpp"

namespace amr {

// Device view of a plan's workspace.
struct DevPlan {
  const InstParams* inst;
  const BlockInfo* blocks;
  const Nbr* nbr;
  const int32_t* fine;
  const int32_t* p2list;
  const int32_t* p2task;  // (leaf, neighbour code) pairs of phase 2: faces, edges, corners
  const int32_t* p2wave;  // phase-2 waves in leaf order: (task row << kP2SubBits) | wave in task
  const int32_t* faceslot;
  const RefluxTask* reflux[3];
  unsigned long long* acc;
  unsigned long long* lacc;  // kCflSlots per leaf: next-step signal-speed maxima of a run of steps
  double* dte;  // per instance: dt / a of a comoving step
  unsigned long long* counters;
  double* ind;
  const MigrTask* migr;
  const Reloc* reloc;
  const int32_t* reloc_child;
  double* faces;
  int64_t nleaf, np2, nreflux[3];
  int64_t np2t[3];  // phase-2 tasks per kind (faces, edges, corners)
  int64_t np2w;     // phase-2 waves
  int32_t p1_large;  // phase-1 refresh of a large mesh: XCD-contiguous order, non-temporal stores
  int32_t ninst, N;
  int32_t nf;  // fields per cell: kFields, or kFieldsDE with the dual-energy field
};

struct LaunchCfg {
  int refresh_block = 256;
  int sweep_block = 256;
  int cfl_block = 256;
  int reflux_block = 256;
  int sweep_mode[3] = {1, 0, 0};  // per axis: 0 = lane-per-pencil walk, 1 = LDS-staged tile
};

hipError_t launch_refresh(const DevPlan& P, double* U, const LaunchCfg& L, hipStream_t st);
// Work items per leaf of the largest forward launch over a plan's leaves
// (a dispatch counts its work items in 32 bits).
int64_t forward_items_per_leaf(int N);
// Refresh of one padded field (per leaf M^3) with unlimited linear
// prolongation into ghosts over a coarser leaf (the composite Poisson
// operator's ghosts).
hipError_t launch_refresh_scalar(const DevPlan& P, double* x, hipStream_t st);
// dt = (C_cfl * a) * min ...; a = 1 outside comoving steps; a_dev (nullable):
// a read on the device instead
hipError_t launch_cfl(const DevPlan& P, const double* U, double* dt, const LaunchCfg& L, hipStream_t st,
                      double a = 1.0, const double* a_dev = nullptr);
// comoving steps (comoving.hip): P.dte = dt / a; the expansion sources with
// rate hubble; a_dev, hubble_dev (nullable): the same read on the device
hipError_t launch_scale_dt(const DevPlan& P, const double* dt, double a, hipStream_t st,
                           const double* a_dev = nullptr);
hipError_t launch_expansion(const DevPlan& P, double* U, const double* dt, double hubble, hipStream_t st,
                            const double* hubble_dev = nullptr);
// transpose of launch_expansion (five fields) at the state U it was applied to
hipError_t launch_expansion_adjoint(const DevPlan& P, const double* U, double* lam, const double* dt, double hubble,
                                   hipStream_t st);
// expansion history on the device (comoving.hip): flat matter + Lambda,
// H(a) = H0 sqrt(om / a^3 + ol), om + ol = 1.  cs = {t, a(t), a(t_mid),
// H(t_mid)}: stage 0 sets cs[1] = a(cs[0]); stage 1, with the step's dt,
// sets t_mid = t + dt / 2, cs[2] = a(t_mid), cs[3] = H(cs[2]), cs[0] = t + dt
hipError_t launch_cosmology(int stage, double H0, double om, double ol, const double* dt, double* cs,
                            hipStream_t st);
// sweep along dir; swept[a] = axis a already swept this step
hipError_t launch_sweep(const DevPlan& P, double* U, const double* dt, int dir, const int swept[3],
                        const LaunchCfg& L, hipStream_t st);
// the same sweep reading Uin and writing every cell of the swept pencils to
// Uout (updated cells, and the others passed through); in place if equal
// cfl_next (in place only): the sweep is a step's last, and its updated cells
// outside the reflux layers add their CFL candidates for the next step to the
// instance accumulators
hipError_t launch_sweep_oop(const DevPlan& P, const double* Uin, double* Uout, const double* dt, int dir,
                            const int swept[3], const LaunchCfg& L, hipStream_t st, int cfl_next = 0);
// after the reflux: the corrected cells' CFL candidates for the next step
hipError_t launch_reflux_cfl(const DevPlan& P, const double* U, hipStream_t st);
// dt = C_cfl * min of the accumulated candidates; resets the accumulators
hipError_t launch_cfl_finalize(const DevPlan& P, double* dt, hipStream_t st);
hipError_t launch_reflux(const DevPlan& P, double* U, const double* dt, int dir, const LaunchCfg& L,
                         hipStream_t st);
// floor-reset counter: mode 0 mark = counter; 1 mark = counter - mark;
// 2 counter = mark
hipError_t launch_floor_mark(const DevPlan& P, unsigned long long* mark, int mode, hipStream_t st);
// per-leaf density-slope indicator into P.ind (needs refreshed ghosts)
hipError_t launch_indicator(const DevPlan& P, const double* U, hipStream_t st);
// counts (bad[0], bad[1]) the operands on which rcp_pos / sqrt_pos differ from
// the IEEE 1/x and sqrt(x); bad is not cleared
hipError_t launch_arith_check(uint64_t seed, int64_t n, unsigned long long* bad, hipStream_t st);
// fill the active cells of every leaf of the new plan P from the old state
hipError_t launch_migrate(const DevPlan& P, const double* Uold, double* Unew, hipStream_t st);

}  // namespace amr
