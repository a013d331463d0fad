// expansion_cell.hpp -- the comoving expansion sources of one active cell
// (paper Sec. II-C: the ppm Method's comoving terms, after Bryan et al.
// 1995), shared by the expansion kernel and the fused kick-and-expansion
// kernels of the comoving self-gravity step, so both round alike.
//
// Crank-Nicolson factors over a time dt with c = (dt / 2) H:
//   m' = m fv,   fv = (1 - c) / (1 + c)
//   ie' = ie fe, fe = (1 - 3 (gamma - 1) c) / (1 + 3 (gamma - 1) c)
//   E' = E + ((ie' - ie) + ke (fv fv - 1))
// where ie = E - ke; an ie' that fell below the pressure floor is raised to
// it, and the dual-energy field rho e takes the same factor and floor rule.
#pragma once

#include "ppm_core.hpp"

namespace amr {

// Updates mx, my, mz, E (and ge when de) in place; returns the number of
// floor resets.
__device__ __forceinline__ unsigned expansion_cell(const InstParams& ip, double c, bool de, double rho, double& mx,
                                                   double& my, double& mz, double& E, double& ge) {
  const double g3 = 3.0 * ip.gm1;
  const double fv = (1.0 - c) / (1.0 + c);
  const double fe = (1.0 - g3 * c) / (1.0 + g3 * c);
  const double ir = rcp_pos(rho);
  const double u = mx * ir, v = my * ir, w = mz * ir;
  const double ke = (0.5 * rho) * ((u * u + v * v) + w * w);
  const double ie = E - ke;
  double ie2 = ie * fe;
  const bool fl = ie2 < ie && ip.gm1 * ie2 < ip.p_floor;
  if (fl) ie2 = ip.p_floor * ip.inv_gm1;
  E = E + ((ie2 - ie) + ke * (fv * fv - 1.0));
  mx = mx * fv;
  my = my * fv;
  mz = mz * fv;
  unsigned n = fl ? 1u : 0u;
  if (de) {
    double ge2 = ge * fe;
    if (ge2 < ge && ip.gm1 * ge2 < ip.p_floor) {
      ge2 = ip.p_floor * ip.inv_gm1;
      n++;
    }
    ge = ge2;
  }
  return n;
}

// Vector-Jacobian product of expansion_cell (five fields) at the cell's
// state before it, with the floor decision held at the forward's (the same
// arithmetic decides it): on entry lr, lm*, lE are the adjoints of rho, the
// momenta and E after the sources, on exit before them.  With ie = E - ke and
// ke = |m|^2 / (2 rho):
//   E' = fe E + (fv^2 - fe) ke   (not floored),   E' = const + fv^2 ke  (floored),
//   m' = fv m,  rho' = rho,  d ke / d m = u,  d ke / d rho = -|u|^2 / 2.
__device__ __forceinline__ void expansion_cell_vjp(const InstParams& ip, double c, double rho, double mx, double my,
                                                   double mz, double E, double& lr, double& lmx, double& lmy,
                                                   double& lmz, double& lE) {
  const double g3 = 3.0 * ip.gm1;
  const double fv = (1.0 - c) / (1.0 + c);
  const double fe = (1.0 - g3 * c) / (1.0 + g3 * c);
  const double ir = rcp_pos(rho);
  const double u = mx * ir, v = my * ir, w = mz * ir;
  const double ke = (0.5 * rho) * ((u * u + v * v) + w * w);
  const double ie = E - ke;
  const double ie2 = ie * fe;
  const bool fl = ie2 < ie && ip.gm1 * ie2 < ip.p_floor;
  const double dk = lE * (fl ? fv * fv : fv * fv - fe);  // adjoint reaching ke
  lr = lr - dk * (0.5 * ((u * u + v * v) + w * w));
  lmx = lmx * fv + dk * u;
  lmy = lmy * fv + dk * v;
  lmz = lmz * fv + dk * w;
  lE = fl ? 0.0 : lE * fe;
}

// The dual-energy field's part: rho e' = fe rho e, or the floor where that
// fell below it (held at the forward's decision).
__device__ __forceinline__ void expansion_ge_vjp(const InstParams& ip, double c, double ge, double& lge) {
  const double g3 = 3.0 * ip.gm1;
  const double fe = (1.0 - g3 * c) / (1.0 + g3 * c);
  const double ge2 = ge * fe;
  lge = (ge2 < ge && ip.gm1 * ge2 < ip.p_floor) ? 0.0 : lge * fe;
}

}  // namespace amr
