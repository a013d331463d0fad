// adjoint.hpp -- launchers of the adjoint kernels (adjoint.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace amr {

// Largest riemann_iters the sweep adjoint supports (its Newton history is
// held in registers).
constexpr int kAdjMaxIters = 8;

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t st);
// reflux transpose: adjoints of the stored face fluxes into gfaces
hipError_t launch_reflux_adjoint(const DevPlan& P, const double* lam, const double* dt, double* gfaces,
                                 hipStream_t st);
// transpose of the sweep along dir whose input state was Uin; floors (device,
// nullable) = post-update floor resets of the forward step: 0 lets the
// kernel skip the floors' products; floors_host = the same count read by the
// host (only the matching kernel is launched), or -1 (not read)
// Work items per leaf of the largest sweep-transpose launch.
int64_t adjoint_items_per_leaf(int N);
hipError_t launch_sweep_adjoint(const DevPlan& P, const double* Uin, double* lam, const double* dt,
                                const double* gfaces, const unsigned long long* floors, int64_t floors_host, int dir,
                                const int swept[3], hipStream_t st);
// transpose of the refresh; Uref = the refreshed state (for the frozen
// prolongation slopes)
hipError_t launch_refresh_adjoint(const DevPlan& P, double* lam, const double* Uref, hipStream_t st);

}  // namespace amr
