// composite.hpp -- launcher of the kernels of mg0 on the octree
// (composite.hip): one call per operation of the composite V-cycle.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace amr {

enum CzKind : int {
  CZ_OPERATOR = 0,   // L = composite operator of the ghost-filled x on colour col (-1: all)
  CZ_UPDATE = 1,     // x -= (b - L) / D on colour col
  CZ_RESID = 2,      // L = b - L
  CZ_RESTRICT = 3,   // b (coarser stage P) = restriction of L (finer stage) by tasks
  CZ_PROLONG = 4,    // x (finer stage P) += interpolation of e (coarser stage, ghosts filled) by tasks
  CZ_COPY_IN = 5,    // x's active cells = src (block layout)
  CZ_COPY_OUT = 6,   // dst (block layout) = x's active cells (minus *scal if scal)
  CZ_ZERO = 7,       // x = 0 (padded, ghosts included)
  CZ_MEAN_SUB = 8,   // b -= scale * volume-weighted sum of b (scale = 1 / weighted volume)
  CZ_MEAN_PADDED = 9,  // scal = scale * volume-weighted sum of x's active cells
  CZ_NORM = 10,      // scal = sqrt(volume-weighted sum of L^2)
  CZ_DENSITY = 11,   // b = fpg * (U's density), active cells
  CZ_KICK = 12,      // half kick of U's active cells with g = -grad(x) (x's ghosts filled), dt on the device
};

struct CzOp {
  int kind = 0;
  DevPlan P{};
  double* x = nullptr;
  double* b = nullptr;
  double* L = nullptr;
  const double* e = nullptr;
  const double* src = nullptr;
  double* dst = nullptr;
  const MigrTask* tasks = nullptr;
  double* parts = nullptr;  // one double per leaf of P
  double* scal = nullptr;
  double scale = 1.0;
  int col = -1;
  double* U = nullptr;        // the hydro state (nf fields of M^3 per leaf)
  const double* dt = nullptr;  // CZ_KICK: the step's dt (device); the kick is (dt/2) scale
  double fpg = 0.0;            // CZ_DENSITY: 4 pi G
};

hipError_t cz_launch(const CzOp& op, hipStream_t st);

}  // namespace amr
