// ppm_core.hpp -- the PPM element formulas of one sweep (paper Sec. II-C,
// the "ppm" Method), written once for the gfx950 kernels and for a host
// build used by the unit tests of the adjoint.  Every formula is evaluated
// exactly as parenthesised; the code is compiled without FMA contraction.
#pragma once
#include <cmath>

#include "layout.hpp"

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define AMR_HD __host__ __device__
#else
#define AMR_HD
#endif

namespace amr {

using std::fabs;
using std::sqrt;

// Reciprocal and square root of an operand in [2^-767, 2^1022] (every
// density, pressure, sound speed and shock mass flux of a step whose floors
// are at least 1e-200).  On the device these are the Newton-Raphson
// reciprocal with Markstein's final correction and the Goldschmidt square
// root, i.e. the IEEE-conforming sequences without their operand scaling and
// special-value fix-ups, which leave such operands unchanged: the results
// are the correctly rounded 1/b and sqrt(x), bit for bit, in fewer
// instructions.
AMR_HD inline double rcp_pos(double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(b);
  double t = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, t, r);
  t = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, t, r);
  t = __builtin_fma(-b, r, 1.0);
  return __builtin_fma(t, r, r);
#else
  return 1.0 / b;
#endif
}
AMR_HD inline double sqrt_pos(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = y * 0.5;
  const double r = __builtin_fma(-h, g, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  double e = __builtin_fma(-g, g, x);
  g = __builtin_fma(e, h, g);
  e = __builtin_fma(-g, g, x);
  return __builtin_fma(e, h, g);
#else
  return sqrt(x);
#endif
}

AMR_HD inline double sel_min(double a, double b) { return a < b ? a : b; }
AMR_HD inline double sel_max(double a, double b) { return a < b ? b : a; }

AMR_HD inline double minmod(double a, double b) {
  return (a * b > 0.0) ? (fabs(a) < fabs(b) ? a : b) : 0.0;
}

struct Par {
  double qL, qR, dq, q6;
};

// MC-limited slope of the middle value.
AMR_HD inline double mc_slope(double qm, double q0, double qp) {
  const double dl = q0 - qm, dr = qp - q0, dc = 0.5 * (qp - qm);
  const double lim = sel_min(sel_min(fabs(dc), 2.0 * fabs(dl)), 2.0 * fabs(dr));
  const double d = dc > 0.0 ? lim : -lim;
  return (dl * dr > 0.0) ? d : 0.0;
}

// Flattened, monotonised parabola of one cell.
AMR_HD inline Par parabola(double q, double qL, double qR, double f, double sixth) {
  qL = f * q + (1.0 - f) * qL;
  qR = f * q + (1.0 - f) * qR;
  Par P;
  if ((qR - q) * (q - qL) <= 0.0) {
    qL = q;
    qR = q;
  } else {
    const double D = qR - qL, mm = q - 0.5 * (qL + qR);
    const double D26 = (D * D) * sixth;
    if (D * mm > D26)
      qL = 3.0 * q - 2.0 * qR;
    else if (-D26 > D * mm)
      qR = 3.0 * q - 2.0 * qL;
  }
  P.qL = qL;
  P.qR = qR;
  P.dq = qR - qL;
  P.q6 = 6.0 * (q - 0.5 * (qL + qR));
  return P;
}

// Mean of the parabola over the fraction s of the cell next to its right
// (Ip) or left (Im) edge.
AMR_HD inline double Ip(const Par& P, double s, double two3) {
  return P.qR - (0.5 * s) * (P.dq - (1.0 - two3 * s) * P.q6);
}
AMR_HD inline double Im(const Par& P, double s, double two3) {
  return P.qL + (0.5 * s) * (P.dq + (1.0 - two3 * s) * P.q6);
}

// Characteristic tracing of one cell (rho, u, c, 1/rho and its 5 parabolas
// in the order rho, u, v, w, p) to the left state at its right edge (WL)
// and the right state at its left edge (WR).
AMR_HD inline void trace(const InstParams& ip, double rho, double u, double c, double ir,
                                      const Par* pa, double nu, double* WL, double* WR) {
  const double two3 = ip.two3;
  const double lm = u - c, l0 = u, lp = u + c;
  const double ic = rcp_pos(c);
  const double Ac = (0.5 * rho) * ic;  // rho / (2c)
  const double Bc = ir * ic;           // 1 / (rho c)
  const double cc = c * c;
  const double ic2 = ic * ic;          // 1 / c^2
  const double cor = c * ir;           // c / rho
  {
    const double sm = (lm > 0.0 ? lm : 0.0) * nu, s0 = (l0 > 0.0 ? l0 : 0.0) * nu, sp = (lp > 0.0 ? lp : 0.0) * nu;
    const double rr = Ip(pa[0], sp, two3), ur = Ip(pa[1], sp, two3), pr = Ip(pa[4], sp, two3);
    const double am = (lm > 0.0) ? Ac * ((pr - Ip(pa[4], sm, two3)) * Bc - (ur - Ip(pa[1], sm, two3))) : 0.0;
    const double a0 = (l0 > 0.0) ? (rr - Ip(pa[0], s0, two3)) - (pr - Ip(pa[4], s0, two3)) * ic2 : 0.0;
    const double r = (rr - am) - a0;
    const double p = pr - cc * am;
    WL[0] = r < ip.rho_floor ? ip.rho_floor : r;
    WL[1] = ur + cor * am;
    WL[2] = Ip(pa[2], s0, two3);
    WL[3] = Ip(pa[3], s0, two3);
    WL[4] = p < ip.p_floor ? ip.p_floor : p;
  }
  {
    const double sm = (lm < 0.0 ? -lm : 0.0) * nu, s0 = (l0 < 0.0 ? -l0 : 0.0) * nu, sp = (lp < 0.0 ? -lp : 0.0) * nu;
    const double rr = Im(pa[0], sm, two3), ur = Im(pa[1], sm, two3), pr = Im(pa[4], sm, two3);
    const double ap = (lp < 0.0) ? Ac * ((pr - Im(pa[4], sp, two3)) * Bc + (ur - Im(pa[1], sp, two3))) : 0.0;
    const double a0 = (l0 < 0.0) ? (rr - Im(pa[0], s0, two3)) - (pr - Im(pa[4], s0, two3)) * ic2 : 0.0;
    const double r = (rr - ap) - a0;
    const double p = pr - cc * ap;
    WR[0] = r < ip.rho_floor ? ip.rho_floor : r;
    WR[1] = ur - cor * ap;
    WR[2] = Im(pa[2], s0, two3);
    WR[3] = Im(pa[3], s0, two3);
    WR[4] = p < ip.p_floor ? ip.p_floor : p;
  }
}

// Pressure before the floor from the total energy E and, with the
// dual-energy field (DE), its internal energy density ge: (gamma-1)(E - ke)
// where E - ke > eta1 E, else (gamma-1) ge; ke = (0.5 rho)((u u + v v) + w w).
template <bool DE>
AMR_HD inline double gas_pressure(const InstParams& ip, double rho, double u, double v, double w, double E,
                                  double ge) {
  const double ie = E - (0.5 * rho) * ((u * u + v * v) + w * w);
  if constexpr (DE) {
    if (!(ie > ip.eta1 * E)) return ip.gm1 * ge;
  }
  return ip.gm1 * ie;
}

// Two-shock Riemann solver (a fixed number of Newton steps on p*, ending
// early only at an exact fixed point, which gives the same bits), sampled at
// x/t = 0, linear fan between head and tail; returns the flux.  Uses the reciprocal
// shock mass fluxes 1/W_K and reciprocal impedances
// 1/Z_K = (1 + (C_K/W_K)^2) / (2 W_K): p* <- p* - (u*_R - u*_L)/(1/Z_L + 1/Z_R).
// DE (dual-energy field): also F[5], the internal-energy flux of the Godunov
// state u_g p_g / (gamma - 1), and *ug = u_g.
template <bool DE = false>
AMR_HD inline void riemann_flux(const InstParams& ip, const double* L, const double* R, double* F,
                                double* ug_out = nullptr) {
  const double rL = L[0], uL = L[1], pL = L[4];
  const double rR = R[0], uR = R[1], pR = R[4];
  const double gam = ip.gamma, g1 = ip.g1, pfl = ip.p_floor;
  const double CL = sqrt_pos((gam * pL) * rL), CR = sqrt_pos((gam * pR) * rR);
  const double ipL = rcp_pos(pL), ipR = rcp_pos(pR);
  double ps = ((CR * pL + CL * pR) - (CL * CR) * (uR - uL)) / (CL + CR);
  ps = ps < pfl ? pfl : ps;
  double WLw, WRw, iWL, iWR, iZL, iZR, usL, usR;
  for (int it = 0;; it++) {
    WLw = CL * sqrt_pos(1.0 + g1 * (ps * ipL - 1.0));
    WRw = CR * sqrt_pos(1.0 + g1 * (ps * ipR - 1.0));
    iWL = rcp_pos(WLw);
    iWR = rcp_pos(WRw);
    usL = uL - (ps - pL) * iWL;
    usR = uR + (ps - pR) * iWR;
    const double qL = CL * iWL, qR = CR * iWR;
    iZL = (0.5 * iWL) * (1.0 + qL * qL);
    iZR = (0.5 * iWR) * (1.0 + qR * qR);
    if (it == ip.iters) break;
    double pn = ps - (usR - usL) / (iZL + iZR);
    pn = pn < pfl ? pfl : pn;
    // a step that leaves p* unchanged has reached a fixed point: every later
    // step would recompute exactly these values, so stopping is exact
    if (pn == ps) break;
    ps = pn;
  }
  const double us = (iZR * usL + iZL * usR) / (iZL + iZR);
  const bool left = us >= 0.0;
  const double s = left ? 1.0 : -1.0;
  const double rK = left ? rL : rR, uK = left ? uL : uR, pK = left ? pL : pR;
  const double WK = left ? WLw : WRw, iWK = left ? iWL : iWR;
  const double irK = rcp_pos(rK);
  const double vs = irK - (ps - pK) * (iWK * iWK);
  const double rs = rcp_pos(vs);
  double rg, ug, pg;
  if (ps > pK) {
    const double S = uK - s * (WK * irK);
    const bool toK = s * S >= 0.0;
    rg = toK ? rK : rs;
    ug = toK ? uK : us;
    pg = toK ? pK : ps;
  } else {
    const double cK = sqrt_pos((gam * pK) * irK);
    const double cs = sqrt_pos((gam * ps) * vs);
    const double lh = uK - s * cK, lt = us - s * cs;
    if (s * lh >= 0.0) {
      rg = rK; ug = uK; pg = pK;
    } else if (s * lt <= 0.0) {
      rg = rs; ug = us; pg = ps;
    } else {
      const double xi = lh / (lh - lt);
      rg = rK + xi * (rs - rK);
      ug = uK + xi * (us - uK);
      pg = pK + xi * (ps - pK);
    }
  }
  const double vg = left ? L[2] : R[2], wg = left ? L[3] : R[3];
  const double mf = rg * ug;
  F[0] = mf;
  F[1] = mf * ug + pg;
  F[2] = mf * vg;
  F[3] = mf * wg;
  F[4] = ug * (pg * ip.g_gm1 + (0.5 * rg) * ((ug * ug + vg * vg) + wg * wg));
  if constexpr (DE) {
    F[5] = ug * (pg * ip.inv_gm1);
    *ug_out = ug;
  }
}


}  // namespace amr
