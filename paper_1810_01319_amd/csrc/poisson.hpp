// poisson.hpp -- the mg0 Poisson solver's launcher (poisson.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace amr {

constexpr int kMgMaxLevels = 24;
constexpr int kMgCoarseMax = 4096;  // cells of the coarsest level (one workgroup's LDS)
constexpr int kMgCoarseSweeps = 64;
// Size of the fixed device buffer that serves as mg_solve's workspace in the
// entry point that allocates nothing: enough for a 128^3 grid (its workspace
// is 38.4 MB).
constexpr int64_t kMgStaticScratchBytes = int64_t(64) << 20;

// Level sizes (x, y, z) of a uniform nx x ny x nz grid: level l+1 halves
// level l while every axis of level l is a multiple of 4.  Returns the count.
int mg_levels(int nx, int ny, int nz, int sizes[][3]);
// Workspace of mg_solve: phi and f of every level (256-byte aligned), then
// the reduction scratch.
int64_t mg_workspace_bytes(int nx, int ny, int nz);
// ncycles V(nu1, nu2) cycles on the uniform periodic grid of the plan's
// level-0 leaves (spacing h), f and phi in the block layout (per leaf N^3
// active cells, x fastest); resid (device, ncycles + 1 doubles) or null.
// f from f_blocks, or (f_blocks null) fpg times the density of the state U.
hipError_t mg_solve(const DevPlan& P, int nx, int ny, int nz, double h, const double* f_blocks, const double* U,
                    double fpg, double* phi_blocks, int ncycles, int nu1, int nu2, double* resid, void* work,
                    hipStream_t st);
// One V(nu1, nu2) cycle from phi = 0 on f (block layout of P's level-0
// leaves), no mean handling; phi into the active cells of x_padded (per leaf
// M^3, one field).  The composite solver's root-level correction.
hipError_t mg_vcycle_blocks(const DevPlan& P, int nx, int ny, int nz, double h, const double* f_blocks,
                            double* x_padded, int nu1, int nu2, void* work, hipStream_t st);
// Half kick of U's active cells with g = -grad(phi) of the mean-free
// potential phi_blocks (block layout), dt from the device: momentum
// + (dt/2) rho g, energy + the kinetic-energy change.
// exp 0: the kick alone; 1: the kick, then the comoving expansion sources
// over *halfdt with expansion rate hubble, in the same pass; 2: the sources,
// then the kick.  level0_current: the workspace's finest level still holds
// phi_blocks' values (the last operation on it was the mg_solve that wrote
// them), so the gather is skipped.
hipError_t mg_kick(const DevPlan& P, int nx, int ny, int nz, double h, double* U, const double* phi_blocks,
                   const double* dt, double scale, void* work, hipStream_t st, int exp = 0,
                   const double* halfdt = nullptr, double hubble = 0.0, bool level0_current = false);
// Device address of the fixed workspace buffer (kMgStaticScratchBytes) on
// the current device, looked up once per device.  Every call on one device
// shares it, so calls that overlap on one device race.
hipError_t mg_static_scratch(void** out);
// Enqueues dt/2 (exact) into a slot of the workspace's scratch and returns
// the slot's device address.
double* mg_half_dt(const double* dt, void* work, int nx, int ny, int nz, hipStream_t st);

}  // namespace amr
