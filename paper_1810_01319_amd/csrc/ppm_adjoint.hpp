// ppm_adjoint.hpp -- vector-Jacobian products of the PPM sweep's formulas
// (ppm_core.hpp), for the hand-written adjoint of a hydro step.
//
// Every discrete branch (slope limiter choice, monotonicity case, flattening
// switch and clamps, wave-direction gates, floors, Riemann side / shock /
// fan) is re-evaluated from the same inputs as the forward and held fixed:
// each function is the exact derivative of the formula on the branch the
// forward took.  The time step is a constant.
#pragma once
#include "ppm_core.hpp"

namespace amr {

// ---- primitives ----------------------------------------------------------

struct Prim {
  double q[5];  // rho, u, v, w, p (floored)
  double c, ir, K;
  bool pfl;     // pressure floor active
  bool sel;     // dual energy: p from the rho e field (E - ke <= eta1 E)
};

AMR_HD inline Prim prim_fwd(const InstParams& ip, const double* U) {
  Prim P;
  P.ir = rcp_pos(U[0]);
  P.q[0] = U[0];
  P.q[1] = U[1] * P.ir;
  P.q[2] = U[2] * P.ir;
  P.q[3] = U[3] * P.ir;
  P.K = (P.q[1] * P.q[1] + P.q[2] * P.q[2]) + P.q[3] * P.q[3];
  const double p = ip.gm1 * (U[4] - (0.5 * U[0]) * P.K);
  P.pfl = p < ip.p_floor;
  P.sel = false;
  P.q[4] = P.pfl ? ip.p_floor : p;
  P.c = sqrt_pos((ip.gamma * P.q[4]) * P.ir);
  return P;
}

// Dual energy: U = (rho, m_n, m_t1, m_t2, E, rho e); the pressure is
// (gamma - 1) rho e where E - ke <= eta1 E (the forward's selection, in its
// arithmetic), else (gamma - 1)(E - ke).
AMR_HD inline Prim prim_fwd_de(const InstParams& ip, const double* U) {
  Prim P;
  P.ir = rcp_pos(U[0]);
  P.q[0] = U[0];
  P.q[1] = U[1] * P.ir;
  P.q[2] = U[2] * P.ir;
  P.q[3] = U[3] * P.ir;
  P.K = (P.q[1] * P.q[1] + P.q[2] * P.q[2]) + P.q[3] * P.q[3];
  const double ie = U[4] - (0.5 * U[0]) * P.K;
  P.sel = !(ie > ip.eta1 * U[4]);
  const double p = P.sel ? ip.gm1 * U[5] : ip.gm1 * ie;
  P.pfl = p < ip.p_floor;
  P.q[4] = P.pfl ? ip.p_floor : p;
  P.c = sqrt_pos((ip.gamma * P.q[4]) * P.ir);
  return P;
}

// g_q[5], g_c, g_ir -> g_U[5] (accumulated); DE: g_U[6], and with the
// selection (P.sel) the pressure's adjoint goes to g_U[5] (rho e) instead
template <bool DE = false>
AMR_HD inline void prim_vjp(const InstParams& ip, const double* U, const Prim& P, const double* gq, double gc,
                            double gir, double* gU) {
  // c = sqrt(gamma p / rho): dc = (gamma / 2c)(dp / rho + p d(1/rho))
  const double h = (0.5 * ip.gamma) * gc / P.c;
  double gp = gq[4] + h * P.ir;
  gir += h * P.q[4];
  if (P.pfl) gp = 0.0;
  double gpm = gp * ip.gm1;
  if constexpr (DE) {
    if (P.sel) {
      gU[5] += gpm;
      gpm = 0.0;
    }
  }
  gU[4] += gpm;
  const double gK = -gpm * (0.5 * U[0]);
  double g0 = gq[0] - gpm * (0.5 * P.K);
  const double gu = gq[1] + gK * (2.0 * P.q[1]);
  const double gv = gq[2] + gK * (2.0 * P.q[2]);
  const double gw = gq[3] + gK * (2.0 * P.q[3]);
  gU[1] += gu * P.ir;
  gU[2] += gv * P.ir;
  gU[3] += gw * P.ir;
  gir += gu * U[1] + gv * U[2] + gw * U[3];
  g0 -= gir * (P.ir * P.ir);
  gU[0] += g0;
}

// ---- MC slope ------------------------------------------------------------

AMR_HD inline void slope_vjp(double qm, double q0, double qp, double g, double* gm, double* g0, double* gp) {
  const double dl = q0 - qm, dr = qp - q0, dc = 0.5 * (qp - qm);
  // every branch sets all three increments and the adds are unconditional,
  // so the accumulators stay in registers (no store through a chosen pointer)
  double em = 0.0, e0 = 0.0, ep = 0.0;
  if (dl * dr > 0.0) {
    const double adc = fabs(dc), a2l = 2.0 * fabs(dl), a2r = 2.0 * fabs(dr);
    const double sg = dc > 0.0 ? 1.0 : -1.0;
    // which term the selects min(min(|dc|, 2|dl|), 2|dr|) returned
    const double m1 = adc < a2l ? adc : a2l;
    if (!(m1 < a2r)) {  // 2|dr|
      const double d = sg * 2.0 * (dr > 0.0 ? 1.0 : -1.0) * g;
      ep = d;
      e0 = -d;
    } else if (adc < a2l) {  // |dc|
      const double d = sg * (dc > 0.0 ? 1.0 : -1.0) * 0.5 * g;
      ep = d;
      em = -d;
    } else {  // 2|dl|
      const double d = sg * 2.0 * (dl > 0.0 ? 1.0 : -1.0) * g;
      e0 = d;
      em = -d;
    }
  }
  *gm += em;
  *g0 += e0;
  *gp += ep;
}

// ---- parabola ------------------------------------------------------------

struct ParGrad {
  double qL, qR, dq, q6;
};

// gradients of the final (qL, qR, dq, q6) -> g of the cell value, of the
// incoming face values and of the flattening coefficient (accumulated)
AMR_HD inline void parabola_vjp(double q, double qLi, double qRi, double f, double sixth, const ParGrad& G,
                                double* gq, double* gqLi, double* gqRi, double* gf) {
  const double qL1 = f * q + (1.0 - f) * qLi;
  const double qR1 = f * q + (1.0 - f) * qRi;
  double gqL = G.qL - G.dq - 3.0 * G.q6;
  double gqR = G.qR + G.dq - 3.0 * G.q6;
  double g_q = 6.0 * G.q6;
  double gqL1 = 0.0, gqR1 = 0.0;
  if ((qR1 - q) * (q - qL1) <= 0.0) {
    g_q += gqL + gqR;
  } else {
    const double D = qR1 - qL1, mm = q - 0.5 * (qL1 + qR1);
    const double D26 = (D * D) * sixth;
    if (D * mm > D26) {
      g_q += 3.0 * gqL;
      gqR1 += gqR - 2.0 * gqL;
    } else if (-D26 > D * mm) {
      g_q += 3.0 * gqR;
      gqL1 += gqL - 2.0 * gqR;
    } else {
      gqL1 += gqL;
      gqR1 += gqR;
    }
  }
  g_q += f * (gqL1 + gqR1);
  *gqLi += (1.0 - f) * gqL1;
  *gqRi += (1.0 - f) * gqR1;
  *gf += gqL1 * (q - qLi) + gqR1 * (q - qRi);
  *gq += g_q;
}

// ---- parabola means ------------------------------------------------------

// Ip(s) = qR - (0.5 s)(dq - (1 - t s) q6)
AMR_HD inline void Ip_vjp(const Par& P, double s, double two3, double g, ParGrad* G, double* gs) {
  G->qR += g;
  G->dq += -(0.5 * s) * g;
  G->q6 += (0.5 * s) * (1.0 - two3 * s) * g;
  *gs += (-0.5 * P.dq + 0.5 * P.q6 - two3 * s * P.q6) * g;
}
// Im(s) = qL + (0.5 s)(dq + (1 - t s) q6)
AMR_HD inline void Im_vjp(const Par& P, double s, double two3, double g, ParGrad* G, double* gs) {
  G->qL += g;
  G->dq += (0.5 * s) * g;
  G->q6 += (0.5 * s) * (1.0 - two3 * s) * g;
  *gs += (0.5 * P.dq + 0.5 * P.q6 - two3 * s * P.q6) * g;
}

// ---- characteristic tracing ----------------------------------------------

// The tracing's coupled part: gWL, gWR (adjoints of the edge states; only
// their rho, u, p entries are used) -> gradients of the rho, u and p
// parabolas (G0, G1, G4) and of rho, u, c, 1/rho of the cell (accumulated).
AMR_HD inline void trace_vjp_rup(const InstParams& ip, double rho, double u, double c, double ir, const Par& p0,
                                 const Par& p1, const Par& p4, double nu, const double* gWL, const double* gWR,
                                 ParGrad* G0, ParGrad* G1, ParGrad* G4, double* grho, double* gu, double* gc,
                                 double* gir) {
  const double t = ip.two3;
  const double lm = u - c, l0 = u, lp = u + c;
  const double ic = rcp_pos(c);
  const double Ac = (0.5 * rho) * ic;
  const double Bc = ir * ic;
  const double cc = c * c;
  const double ic2 = ic * ic;
  const double cor = c * ir;
  double gAc = 0, gBc = 0, gcc = 0, gic2 = 0, gcor = 0, glm = 0, gl0 = 0, glp = 0;
  // ---- right edge (left state at j+1/2) ----
  {
    const double sm = (lm > 0.0 ? lm : 0.0) * nu, s0 = (l0 > 0.0 ? l0 : 0.0) * nu, sp = (lp > 0.0 ? lp : 0.0) * nu;
    const double rr = Ip(p0, sp, t), ur = Ip(p1, sp, t), pr = Ip(p4, sp, t);
    const double Ipm = Ip(p4, sm, t), Ium = Ip(p1, sm, t);
    const double Ir0 = Ip(p0, s0, t), Ip0 = Ip(p4, s0, t);
    const double X = pr - Ipm, Y = ur - Ium;
    const double am = (lm > 0.0) ? Ac * (X * Bc - Y) : 0.0;
    const double a0 = (l0 > 0.0) ? (rr - Ir0) - (pr - Ip0) * ic2 : 0.0;
    const double r = (rr - am) - a0;
    const double p = pr - cc * am;
    const double g0 = r < ip.rho_floor ? 0.0 : gWL[0];
    const double g4 = p < ip.p_floor ? 0.0 : gWL[4];
    double grr = g0, gur = gWL[1], gpr = g4;
    double gam = -g0 + cor * gWL[1] - cc * g4;
    const double ga0 = -g0;
    gcor += gWL[1] * am;
    gcc += -g4 * am;
    double gsm = 0, gs0 = 0, gsp = 0;
    if (l0 > 0.0) {
      grr += ga0;
      Ip_vjp(p0, s0, t, -ga0, G0, &gs0);
      gpr -= ga0 * ic2;
      Ip_vjp(p4, s0, t, ga0 * ic2, G4, &gs0);
      gic2 -= ga0 * (pr - Ip0);
    }
    if (lm > 0.0) {
      gAc += gam * (X * Bc - Y);
      const double gX = gam * Ac * Bc, gY = -gam * Ac;
      gBc += gam * Ac * X;
      gpr += gX;
      Ip_vjp(p4, sm, t, -gX, G4, &gsm);
      gur += gY;
      Ip_vjp(p1, sm, t, -gY, G1, &gsm);
    }
    Ip_vjp(p0, sp, t, grr, G0, &gsp);
    Ip_vjp(p1, sp, t, gur, G1, &gsp);
    Ip_vjp(p4, sp, t, gpr, G4, &gsp);
    if (lm > 0.0) glm += nu * gsm;
    if (l0 > 0.0) gl0 += nu * gs0;
    if (lp > 0.0) glp += nu * gsp;
  }
  // ---- left edge (right state at j-1/2) ----
  {
    const double sm = (lm < 0.0 ? -lm : 0.0) * nu, s0 = (l0 < 0.0 ? -l0 : 0.0) * nu, sp = (lp < 0.0 ? -lp : 0.0) * nu;
    const double rr = Im(p0, sm, t), ur = Im(p1, sm, t), pr = Im(p4, sm, t);
    const double Imp = Im(p4, sp, t), Imu = Im(p1, sp, t);
    const double Ir0 = Im(p0, s0, t), Ip0 = Im(p4, s0, t);
    const double X = pr - Imp, Y = ur - Imu;
    const double ap = (lp < 0.0) ? Ac * (X * Bc + Y) : 0.0;
    const double a0 = (l0 < 0.0) ? (rr - Ir0) - (pr - Ip0) * ic2 : 0.0;
    const double r = (rr - ap) - a0;
    const double p = pr - cc * ap;
    const double g0 = r < ip.rho_floor ? 0.0 : gWR[0];
    const double g4 = p < ip.p_floor ? 0.0 : gWR[4];
    double grr = g0, gur = gWR[1], gpr = g4;
    const double gap = -g0 - cor * gWR[1] - cc * g4;
    const double ga0 = -g0;
    gcor += -gWR[1] * ap;
    gcc += -g4 * ap;
    double gsm = 0, gs0 = 0, gsp = 0;
    if (l0 < 0.0) {
      grr += ga0;
      Im_vjp(p0, s0, t, -ga0, G0, &gs0);
      gpr -= ga0 * ic2;
      Im_vjp(p4, s0, t, ga0 * ic2, G4, &gs0);
      gic2 -= ga0 * (pr - Ip0);
    }
    if (lp < 0.0) {
      gAc += gap * (X * Bc + Y);
      const double gX = gap * Ac * Bc, gY = gap * Ac;
      gBc += gap * Ac * X;
      gpr += gX;
      Im_vjp(p4, sp, t, -gX, G4, &gsp);
      gur += gY;
      Im_vjp(p1, sp, t, -gY, G1, &gsp);
    }
    Im_vjp(p0, sm, t, grr, G0, &gsm);
    Im_vjp(p1, sm, t, gur, G1, &gsm);
    Im_vjp(p4, sm, t, gpr, G4, &gsm);
    if (lm < 0.0) glm -= nu * gsm;
    if (l0 < 0.0) gl0 -= nu * gs0;
    if (lp < 0.0) glp -= nu * gsp;
  }
  // ---- common quantities ----
  double gic = gAc * (0.5 * rho) + gBc * ir + gic2 * (2.0 * ic);
  *grho += gAc * (0.5 * ic);
  *gir += gBc * ic + gcor * c;
  double g_c = gcc * (2.0 * c) + gcor * ir - gic * (ic * ic);
  *gu += glm + gl0 + glp;
  g_c += -glm + glp;
  *gc += g_c;
}

// A transverse field of the tracing (v or w): its edge states are the
// parabola's means over the entropy wave's reach, WL_t = Ip(s0) at j+1/2 and
// WR_t = Im(s0') at j-1/2 -> gradient of its parabola and of u (accumulated).
AMR_HD inline void trace_vjp_transverse(double u, double nu, double two3, const Par& pa, double gWLt, double gWRt,
                                        ParGrad* G, double* gu) {
  const double sR = (u > 0.0 ? u : 0.0) * nu, sL = (u < 0.0 ? -u : 0.0) * nu;
  double gsR = 0, gsL = 0;
  Ip_vjp(pa, sR, two3, gWLt, G, &gsR);
  Im_vjp(pa, sL, two3, gWRt, G, &gsL);
  if (u > 0.0) *gu += nu * gsR;
  if (u < 0.0) *gu -= nu * gsL;
}

// The whole tracing: gWL, gWR -> gradients of the 5 parabolas and of rho, u,
// c, 1/rho of the cell (accumulated).
AMR_HD inline void trace_vjp(const InstParams& ip, double rho, double u, double c, double ir, const Par* pa, double nu,
                             const double* gWL, const double* gWR, ParGrad* G, double* grho, double* gu, double* gc,
                             double* gir) {
  trace_vjp_rup(ip, rho, u, c, ir, pa[0], pa[1], pa[4], nu, gWL, gWR, &G[0], &G[1], &G[4], grho, gu, gc, gir);
  trace_vjp_transverse(u, nu, ip.two3, pa[2], gWL[2], gWR[2], &G[2], gu);
  trace_vjp_transverse(u, nu, ip.two3, pa[3], gWL[3], gWR[3], &G[3], gu);
}

// ---- two-shock Riemann solver -------------------------------------------

// gF (flux) -> gL, gR (edge states rho,u,v,w,p; accumulated).  MAXIT bounds
// ip.iters at compile time: with the loops unrolled the Newton history stays
// in registers.  The forward part repeats riemann_flux's arithmetic exactly
// (same branches); the reverse part evaluates each Newton evaluation's square
// roots and reciprocals once and shares reciprocals between the derivative
// terms.
// FIXSTOP = false reverses every evaluation one by one (a host-side check of
// the closed form used at a fixed point).
// DE: also the adjoints of the rho e flux F[5] = u_g p_g / (gamma - 1)
// (gF5) and of the Godunov velocity u_g itself (gUg).
template <int MAXIT, bool FIXSTOP = true, bool DE = false>
AMR_HD inline void riemann_vjp_n(const InstParams& ip, const double* L, const double* R, const double* gF, double* gL,
                                 double* gR, double gF5 = 0.0, double gUg = 0.0) {
  const double rL = L[0], uL = L[1], pL = L[4];
  const double rR = R[0], uR = R[1], pR = R[4];
  const double gam = ip.gamma, g1 = ip.g1, pfl = ip.p_floor;
  const int NI = ip.iters;
  // ---- forward, keeping p* of every Newton evaluation ----
  const double CL = sqrt_pos((gam * pL) * rL), CR = sqrt_pos((gam * pR) * rR);
  const double ipL = rcp_pos(pL), ipR = rcp_pos(pR);
  const double num0 = (CR * pL + CL * pR) - (CL * CR) * (uR - uL);
  const double den0 = CL + CR;
  double ps = num0 / den0;
  const bool fl0 = ps < pfl;
  ps = fl0 ? pfl : ps;
  double psv[MAXIT + 1];
  bool flv[MAXIT + 1];
  double WLw = 0, WRw = 0, iWL = 0, iWR = 0, iZL = 0, iZR = 0, usL = 0, usR = 0, sLf = 1, sRf = 1;
  // evaluations kfix..NI all take place at the same p* once a Newton step
  // leaves p* unchanged (a fixed point: the forward stops there with the
  // same bits); their reverse is done in closed form below
  int kfix = NI;
#pragma unroll
  for (int it = 0; it <= MAXIT; it++) {
    psv[it] = ps;
    sLf = sqrt_pos(1.0 + g1 * (ps * ipL - 1.0));
    sRf = sqrt_pos(1.0 + g1 * (ps * ipR - 1.0));
    WLw = CL * sLf;
    WRw = CR * sRf;
    iWL = rcp_pos(WLw);
    iWR = rcp_pos(WRw);
    usL = uL - (ps - pL) * iWL;
    usR = uR + (ps - pR) * iWR;
    const double qL = CL * iWL, qR = CR * iWR;
    iZL = (0.5 * iWL) * (1.0 + qL * qL);
    iZR = (0.5 * iWR) * (1.0 + qR * qR);
    if (it == NI) break;
    double pn = ps - (usR - usL) / (iZL + iZR);
    flv[it] = pn < pfl;
    pn = flv[it] ? pfl : pn;
    if (FIXSTOP && pn == ps) {
      kfix = it;
      break;
    }
    ps = pn;
  }
  const double Dz = iZL + iZR;
  const double us = (iZR * usL + iZL * usR) / Dz;
  const bool left = us >= 0.0;
  const double s = left ? 1.0 : -1.0;
  const double rK = left ? rL : rR, uK = left ? uL : uR, pK = left ? pL : pR;
  const double WK = left ? WLw : WRw, iWK = left ? iWL : iWR;
  const double irK = rcp_pos(rK);
  const double vs = irK - (ps - pK) * (iWK * iWK);
  const double rs = rcp_pos(vs);
  // sampled state and its case: 0 = side state, 1 = star, 2 = fan
  int cse;
  double xi = 0, lh = 0, lt = 0, cK = 0, csr = 0;
  if (ps > pK) {
    const double S = uK - s * (WK * irK);
    cse = (s * S >= 0.0) ? 0 : 1;
  } else {
    cK = sqrt_pos((gam * pK) * irK);
    csr = sqrt_pos((gam * ps) * vs);
    lh = uK - s * cK;
    lt = us - s * csr;
    if (s * lh >= 0.0) cse = 0;
    else if (s * lt <= 0.0) cse = 1;
    else {
      cse = 2;
      xi = lh / (lh - lt);
    }
  }
  double rg, ug, pg;
  if (cse == 0) { rg = rK; ug = uK; pg = pK; }
  else if (cse == 1) { rg = rs; ug = us; pg = ps; }
  else { rg = rK + xi * (rs - rK); ug = uK + xi * (us - uK); pg = pK + xi * (ps - pK); }
  const double vg = left ? L[2] : R[2], wg = left ? L[3] : R[3];
  const double mf = rg * ug;
  const double K2 = (ug * ug + vg * vg) + wg * wg;
  const double H = pg * ip.g_gm1 + (0.5 * rg) * K2;
  // ---- reverse: flux ----
  const double gmf = gF[0] + gF[1] * ug + gF[2] * vg + gF[3] * wg;
  double gug = gF[1] * mf + gF[4] * H;
  const double gH = gF[4] * ug;
  double gpg = gF[1] + gH * ip.g_gm1;
  double grg = gH * (0.5 * K2);
  const double gK2 = gH * (0.5 * rg);
  gug += gK2 * (2.0 * ug);
  const double gvg = gF[2] * mf + gK2 * (2.0 * vg);
  const double gwg = gF[3] * mf + gK2 * (2.0 * wg);
  grg += gmf * ug;
  gug += gmf * rg;
  if constexpr (DE) {
    gug += gF5 * (pg * ip.inv_gm1) + gUg;
    gpg += (gF5 * ug) * ip.inv_gm1;
  }
  if (left) { gL[2] += gvg; gL[3] += gwg; }
  else { gR[2] += gvg; gR[3] += gwg; }
  // ---- reverse: sampling ----
  double grK = 0, guK = 0, gpK = 0, grs = 0, gus = 0, gps = 0, gvs = 0, girK = 0, giWK = 0;
  if (cse == 0) { grK += grg; guK += gug; gpK += gpg; }
  else if (cse == 1) { grs += grg; gus += gug; gps += gpg; }
  else {
    grK += grg * (1.0 - xi); grs += grg * xi;
    guK += gug * (1.0 - xi); gus += gug * xi;
    gpK += gpg * (1.0 - xi); gps += gpg * xi;
    const double gxi = grg * (rs - rK) + gug * (us - uK) + gpg * (ps - pK);
    const double d = lh - lt;
    const double gxd = gxi / (d * d);
    const double glh = -gxd * lt, glt = gxd * lh;
    guK += glh;
    const double gcK = -s * glh;
    gus += glt;
    const double gcs = -s * glt;
    // c = sqrt(gam p / rho): dc = (gam / 2c) (dp / rho + p d(1/rho))
    const double hK = (0.5 * gam) * gcK / cK, hs = (0.5 * gam) * gcs / csr;
    gpK += hK * irK;
    girK += hK * pK;
    gps += hs * vs;
    gvs += hs * ps;
  }
  gvs += -grs * (rs * rs);
  girK += gvs;
  const double iWK2 = iWK * iWK;
  gps += -gvs * iWK2;
  gpK += gvs * iWK2;
  giWK += -gvs * (ps - pK) * (2.0 * iWK);
  grK += -girK * (irK * irK);
  // star velocity u* = (iZR usL + iZL usR) / (iZL + iZR)
  const double iDz = rcp_pos(Dz);
  double gusL = gus * iZR * iDz, gusR = gus * iZL * iDz;
  double giZR = gus * (usL - us) * iDz, giZL = gus * (usR - us) * iDz;
  double giWL = left ? giWK : 0.0, giWR = left ? 0.0 : giWK;
  // side-K inputs
  double grL = 0, guL = 0, gpL = 0, grR = 0, guR = 0, gpR = 0;
  if (left) { grL += grK; guL += guK; gpL += gpK; }
  else { grR += grK; guR += guK; gpR += gpK; }
  // ---- reverse through the Newton evaluations, last first ----
  // Evaluation at p: s = sqrt(1 + g1 (p/pK - 1)), 1/W = 1/(C s), q = C/W,
  // 1/Z = (1/(2W))(1 + q^2), u*_K = u_K -+ (p - p_K)/W_K.
  double gCL = 0, gCR = 0, gipL = 0, gipR = 0;
  double gps_cur = gps;  // adjoint of the p* the evaluation being reversed used
  double sl = sLf, sr = sRf, iwl = iWL, iwr = iWR;  // that evaluation's values
  // reverse of one evaluation at p (inputs giZL, giZR, gusL, gusR, giWL,
  // giWR; output added to gps_cur and the accumulators)
  auto eval_rev = [&](double p) {
    const double ql = CL * iwl, qr = CR * iwr;
    giWL += giZL * (0.5 * (1.0 + ql * ql));
    const double gql = giZL * (iwl * ql);
    giWR += giZR * (0.5 * (1.0 + qr * qr));
    const double gqr = giZR * (iwr * qr);
    gCL += gql * iwl;
    giWL += gql * CL;
    gCR += gqr * iwr;
    giWR += gqr * CR;
    guL += gusL;
    gps_cur += -gusL * iwl;
    gpL += gusL * iwl;
    giWL += -gusL * (p - pL);
    guR += gusR;
    gps_cur += gusR * iwr;
    gpR += -gusR * iwr;
    giWR += gusR * (p - pR);
    // W = C s: dW = s dC + C ds; ds = g1 da / (2 s) with 1/s = C/W
    const double gWl = -giWL * (iwl * iwl), gWr = -giWR * (iwr * iwr);
    gCL += gWl * sl;
    gCR += gWr * sr;
    const double gaL = (0.5 * g1) * gWl * (CL * CL * iwl), gaR = (0.5 * g1) * gWr * (CR * CR * iwr);
    gps_cur += gaL * ipL + gaR * ipR;
    gipL += gaL * p;
    gipR += gaR * p;
  };
  // reverse of the Newton update p = p_prev - (u*_R - u*_L) / (1/Z_L + 1/Z_R)
  // into the evaluation at p_prev (whose values are in sl, sr, iwl, iwr)
  auto update_rev = [&](double pp, bool floored) {
    double gprev = 0.0;
    giZL = giZR = gusL = gusR = giWL = giWR = 0.0;
    if (!floored) {
      const double uls = uL - (pp - pL) * iwl, urs = uR + (pp - pR) * iwr;
      const double zl = (0.5 * iwl) * (1.0 + (CL * iwl) * (CL * iwl));
      const double zr = (0.5 * iwr) * (1.0 + (CR * iwr) * (CR * iwr));
      const double iD = rcp_pos(zl + zr);
      const double gD = gps_cur * iD;
      gprev = gps_cur;
      gusR = -gD;
      gusL = gD;
      giZL = giZR = gD * (urs - uls) * iD;
    }
    gps_cur = gprev;
  };
  eval_rev(ps);  // the last evaluation (at the final p*, psv[kfix] = ... = psv[NI])
  if (kfix < NI) {
    // m = NI - kfix identical (update, evaluation) pairs at p*: each maps the
    // adjoint g of p* to J g and adds g a to the accumulators (a, J constants
    // at p*).  One pair run with g (1 + J + ... + J^(m-1)) adds exactly the m
    // pairs' sum; the adjoint leaving them is J^m g.
    const double p = ps;
    const int m = NI - kfix;
    double J = 0.0;
    if (!flv[kfix]) {
      const double uls = usL, urs = usR;
      const double iD = rcp_pos(iZL + iZR);
      const double z = (urs - uls) * iD * iD;  // giZ per unit g
      const double ql = CL * iwl, qr = CR * iwr;
      const double wl = z * (0.5 * (1.0 + ql * ql)) + z * (iwl * ql) * CL - iD * (p - pL);
      const double wr = z * (0.5 * (1.0 + qr * qr)) + z * (iwr * qr) * CR - iD * (p - pR);
      const double aL = (0.5 * g1) * (-wl * (iwl * iwl)) * (CL * CL * iwl);
      const double aR = (0.5 * g1) * (-wr * (iwr * iwr)) * (CR * CR * iwr);
      J = 1.0 + ((-iD * iwl - iD * iwr) + (aL * ipL + aR * ipR));
    }
    double S = 0.0, Jm = 1.0;
#pragma unroll
    for (int i = 0; i < MAXIT; i++) {
      if (i < m) {
        S += Jm;
        Jm *= J;
      }
    }
    const double g = gps_cur;
    gps_cur = g * S;
    update_rev(p, flv[kfix]);
    eval_rev(p);
    gps_cur = g * Jm;
  }
  // the evaluations before the fixed point, last first
#pragma unroll
  for (int it = MAXIT; it >= 1; it--) {
    if (it > kfix) continue;
    const double pp = psv[it - 1];
    sl = sqrt_pos(1.0 + g1 * (pp * ipL - 1.0));
    sr = sqrt_pos(1.0 + g1 * (pp * ipR - 1.0));
    iwl = rcp_pos(CL * sl);
    iwr = rcp_pos(CR * sr);
    update_rev(pp, flv[it - 1]);
    eval_rev(pp);
  }
  // first guess p* = num0 / den0 (unless floored)
  if (!fl0) {
    const double gnum = gps_cur / den0;
    const double gden = -gnum * (num0 / den0);
    gCR += gnum * (pL - CL * (uR - uL)) + gden;
    gCL += gnum * (pR - CR * (uR - uL)) + gden;
    gpL += gnum * CR;
    gpR += gnum * CL;
    guR += -gnum * (CL * CR);
    guL += gnum * (CL * CR);
  }
  gpL += -gipL * (ipL * ipL);
  gpR += -gipR * (ipR * ipR);
  // C = sqrt(gam p rho): dC = (gam / 2C)(rho dp + p drho)
  const double hL = (0.5 * gam) * gCL / CL, hR = (0.5 * gam) * gCR / CR;
  gpL += hL * rL;
  grL += hL * pL;
  gpR += hR * rR;
  grR += hR * pR;
  gL[0] += grL; gL[1] += guL; gL[4] += gpL;
  gR[0] += grR; gR[1] += guR; gR[4] += gpR;
}

AMR_HD inline void riemann_vjp(const InstParams& ip, const double* L, const double* R, const double* gF, double* gL,
                               double* gR) {
  riemann_vjp_n<64>(ip, L, R, gF, gL, gR);
}

// ---- post-update floors ----------------------------------------------------

// The floors the update applies to a cell's new conserved values V (pencil
// roles rho, m_n, m_t1, m_t2, E): rho is raised to the density floor, then E
// is reset to the floor pressure's energy if the pressure fell below it.
AMR_HD inline void floor_apply(const InstParams& ip, const double* V, double* out) {
  double r0 = V[0];
  if (r0 < ip.rho_floor) r0 = ip.rho_floor;
  const double jr = rcp_pos(r0);
  const double a1 = V[1] * jr, a2 = V[2] * jr, a3 = V[3] * jr;
  const double ke = (0.5 * r0) * ((a1 * a1 + a2 * a2) + a3 * a3);
  double e = V[4];
  if (ip.gm1 * (e - ke) < ip.p_floor) e = ip.p_floor * ip.inv_gm1 + ke;
  out[0] = r0;
  out[1] = V[1];
  out[2] = V[2];
  out[3] = V[3];
  out[4] = e;
}

// g (adjoint of the floored values) -> gV (adjoint of V); may alias g.
// With the pressure floor active E = const + |m|^2 / (2 rho).
AMR_HD inline void floor_vjp(const InstParams& ip, const double* V, const double* g, double* gV) {
  const bool rfl = V[0] < ip.rho_floor;
  const double r0 = rfl ? ip.rho_floor : V[0];
  const double jr = rcp_pos(r0);
  const double a1 = V[1] * jr, a2 = V[2] * jr, a3 = V[3] * jr;
  const double K = (a1 * a1 + a2 * a2) + a3 * a3;
  const double ke = (0.5 * r0) * K;
  const bool pfl = ip.gm1 * (V[4] - ke) < ip.p_floor;
  const double g4 = g[4];
  double gr = g[0];
  if (pfl) {
    gV[1] = g[1] + g4 * a1;
    gV[2] = g[2] + g4 * a2;
    gV[3] = g[3] + g4 * a3;
    gr += -0.5 * K * g4;
    gV[4] = 0.0;
  } else {
    gV[1] = g[1];
    gV[2] = g[2];
    gV[3] = g[3];
    gV[4] = g4;
  }
  gV[0] = rfl ? 0.0 : gr;
}

// Dual energy: the update's floors and resynchronisation of one cell.  V
// holds the pre-floor values (rho, m_n, m_t1, m_t2, E, rho e), rho e already
// with its flux difference and work term.  Forward: the density and pressure
// floors as floor_apply, then rho e takes E - ke where E - ke > eta2 E, then
// its own floor (gamma - 1) rho e >= p_floor.
AMR_HD inline void floor_apply_de(const InstParams& ip, const double* V, double* out) {
  floor_apply(ip, V, out);
  const double jr = rcp_pos(out[0]);
  const double a1 = V[1] * jr, a2 = V[2] * jr, a3 = V[3] * jr;
  const double ke = (0.5 * out[0]) * ((a1 * a1 + a2 * a2) + a3 * a3);
  double ge = V[5];
  const double ie = out[4] - ke;
  if (ie > ip.eta2 * out[4]) ge = ie;
  if (ip.gm1 * ge < ip.p_floor) ge = ip.p_floor * ip.inv_gm1;
  out[5] = ge;
}

// g (adjoint of the six outputs) -> gV (adjoint of V); may alias g.
AMR_HD inline void floor_vjp_de(const InstParams& ip, const double* V, const double* g, double* gV) {
  const bool rfl = V[0] < ip.rho_floor;
  const double r0 = rfl ? ip.rho_floor : V[0];
  const double jr = rcp_pos(r0);
  const double a1 = V[1] * jr, a2 = V[2] * jr, a3 = V[3] * jr;
  const double K = (a1 * a1 + a2 * a2) + a3 * a3;
  const double ke = (0.5 * r0) * K;
  const bool pfl = ip.gm1 * (V[4] - ke) < ip.p_floor;
  const double e = pfl ? ip.p_floor * ip.inv_gm1 + ke : V[4];
  const double ie = e - ke;
  const bool rsy = ie > ip.eta2 * e;
  const double ge = rsy ? ie : V[5];
  const bool gfl = ip.gm1 * ge < ip.p_floor;
  const double g5 = gfl ? 0.0 : g[5];
  // rho e = E - ke (resynchronised) passes g5 to E and -g5 to ke
  const double gE = g[4] + (rsy ? g5 : 0.0);
  double gke = rsy ? -g5 : 0.0;
  gV[5] = rsy ? 0.0 : g5;
  // the pressure floor: E = const + ke
  if (pfl) {
    gke += gE;
    gV[4] = 0.0;
  } else {
    gV[4] = gE;
  }
  // ke = |m|^2 / (2 rho): d/dm = a, d/drho = -K / 2
  const double gr = g[0] - (0.5 * K) * gke;
  gV[1] = g[1] + gke * a1;
  gV[2] = g[2] + gke * a2;
  gV[3] = g[3] + gke * a3;
  gV[0] = rfl ? 0.0 : gr;
}

// ---- one pencil ------------------------------------------------------------

constexpr int kMaxPencil = 38;

// Adjoint of one pencil's sweep update.  U: the sweep's input cells
// (pencil roles rho, m_n, m_t1, m_t2, E) as U[v * n + j]; lam: on entry the
// adjoint of the sweep's output on the same cells, on exit the adjoint of
// its input (cells outside [lo, hi) are not updated by the sweep and keep
// their identity part).  gface_lo/hi: adjoints of the fluxes at j = lo-1/2
// and hi-1/2 stored for reflux (nullptr if none).  Reference composition for
// the host tests: the gfx950 kernel applies the same element products in
// LDS-staged phases.
AMR_HD inline void pencil_vjp(const InstParams& ip, double nu, int n, int lo, int hi, const double* U, double* lam,
                              const double* gface_lo, const double* gface_hi) {
  Prim P[kMaxPencil];
  double dl[kMaxPencil][5], fa[kMaxPencil][5], fl[kMaxPencil];
  Par pa[kMaxPencil][5];
  double WL[kMaxPencil][5], WR[kMaxPencil][5];
  const double sixth = ip.sixth;
  for (int j = 0; j < n; j++) {
    double u5[5] = {U[j], U[n + j], U[2 * n + j], U[3 * n + j], U[4 * n + j]};
    P[j] = prim_fwd(ip, u5);
  }
  for (int j = 1; j <= n - 2; j++)
    for (int v = 0; v < 5; v++) dl[j][v] = mc_slope(P[j - 1].q[v], P[j].q[v], P[j + 1].q[v]);
  for (int j = 1; j <= n - 3; j++)
    for (int v = 0; v < 5; v++)
      fa[j][v] = 0.5 * (P[j].q[v] + P[j + 1].q[v]) - (dl[j + 1][v] - dl[j][v]) * sixth;
  bool shk[kMaxPencil], fact[kMaxPencil];
  double rr_[kMaxPencil];
  for (int j = 2; j <= n - 3; j++) {
    const double pp1 = P[j + 1].q[4], pm1 = P[j - 1].q[4];
    const double dp1 = pp1 - pm1;
    const double pmin = pp1 < pm1 ? pp1 : pm1;
    shk[j] = (fabs(dp1) > 0.33 * pmin) && (P[j - 1].q[1] - P[j + 1].q[1] > 0.0);
    const double dp2 = P[j + 2].q[4] - P[j - 2].q[4];
    const double r = (dp2 != 0.0) ? dp1 / dp2 : 0.0;
    rr_[j] = r;
    double ft = 10.0 * (r - 0.75);
    fact[j] = shk[j] && dp2 != 0.0 && ft < 1.0 && ft > 0.0;
    ft = ft < 1.0 ? ft : 1.0;
    ft = ft > 0.0 ? ft : 0.0;
    fl[j] = shk[j] ? ft : 0.0;
    for (int v = 0; v < 5; v++) pa[j][v] = parabola(P[j].q[v], fa[j - 1][v], fa[j][v], fl[j], sixth);
    trace(ip, P[j].q[0], P[j].q[1], P[j].c, P[j].ir, pa[j], nu, WL[j], WR[j]);
  }
  // adjoint accumulators
  double gq[kMaxPencil][5] = {}, gc[kMaxPencil] = {}, gir[kMaxPencil] = {};
  double gdl[kMaxPencil][5] = {}, gfa[kMaxPencil][5] = {}, gfl[kMaxPencil] = {};
  double gWL[kMaxPencil][5] = {}, gWR[kMaxPencil][5] = {};
  // update U_j -= nu (F_{j+1/2} - F_{j-1/2}) on [lo, hi), then floors: the
  // adjoint of the pre-floor values replaces lam there
  for (int j = lo; j < hi; j++) {
    double F0[5], F1[5], V[5], g[5];
    riemann_flux(ip, WL[j - 1], WR[j], F0);
    riemann_flux(ip, WL[j], WR[j + 1], F1);
    for (int v = 0; v < 5; v++) {
      V[v] = U[v * n + j] - nu * (F1[v] - F0[v]);
      g[v] = lam[v * n + j];
    }
    floor_vjp(ip, V, g, g);
    for (int v = 0; v < 5; v++) lam[v * n + j] = g[v];
  }
  // faces for reflux
  for (int j = lo - 1; j <= hi - 1; j++) {
    double gF[5];
    for (int v = 0; v < 5; v++) {
      const double up = (j + 1 >= lo && j + 1 < hi) ? lam[v * n + j + 1] : 0.0;
      const double dn = (j >= lo && j < hi) ? lam[v * n + j] : 0.0;
      gF[v] = nu * (up - dn);
    }
    if (j == lo - 1 && gface_lo)
      for (int v = 0; v < 5; v++) gF[v] += gface_lo[v];
    if (j == hi - 1 && gface_hi)
      for (int v = 0; v < 5; v++) gF[v] += gface_hi[v];
    riemann_vjp(ip, WL[j], WR[j + 1], gF, gWL[j], gWR[j + 1]);
  }
  for (int j = 2; j <= n - 3; j++) {
    ParGrad G[5] = {};
    double grho = 0, gu = 0;
    trace_vjp(ip, P[j].q[0], P[j].q[1], P[j].c, P[j].ir, pa[j], nu, gWL[j], gWR[j], G, &grho, &gu, &gc[j], &gir[j]);
    gq[j][0] += grho;
    gq[j][1] += gu;
    for (int v = 0; v < 5; v++)
      parabola_vjp(P[j].q[v], fa[j - 1][v], fa[j][v], fl[j], sixth, G[v], &gq[j][v], &gfa[j - 1][v], &gfa[j][v],
                   &gfl[j]);
    if (fact[j]) {
      const double gr = 10.0 * gfl[j];
      const double dp2 = P[j + 2].q[4] - P[j - 2].q[4];
      const double gdp1 = gr / dp2, gdp2 = -gr * rr_[j] / dp2;
      gq[j + 1][4] += gdp1;
      gq[j - 1][4] -= gdp1;
      gq[j + 2][4] += gdp2;
      gq[j - 2][4] -= gdp2;
    }
  }
  for (int j = 1; j <= n - 3; j++)
    for (int v = 0; v < 5; v++) {
      const double g = gfa[j][v];
      gq[j][v] += 0.5 * g;
      gq[j + 1][v] += 0.5 * g;
      gdl[j + 1][v] -= sixth * g;
      gdl[j][v] += sixth * g;
    }
  for (int j = 1; j <= n - 2; j++)
    for (int v = 0; v < 5; v++)
      slope_vjp(P[j - 1].q[v], P[j].q[v], P[j + 1].q[v], gdl[j][v], &gq[j - 1][v], &gq[j][v], &gq[j + 1][v]);
  for (int j = 0; j < n; j++) {
    double u5[5] = {U[j], U[n + j], U[2 * n + j], U[3 * n + j], U[4 * n + j]};
    double gU[5] = {0, 0, 0, 0, 0};
    prim_vjp(ip, u5, P[j], gq[j], gc[j], gir[j], gU);
    for (int v = 0; v < 5; v++) lam[v * n + j] += gU[v];
  }
}


// Dual energy: the same with the sixth field rho e (U, lam and the face
// adjoints carry six fields).  rho e enters the sweep through the pressure
// selection of the primitives, its flux u_g p_g / (gamma - 1) and the work
// term of the update; the update's floors and resynchronisation follow
// floor_vjp_de.
AMR_HD inline void pencil_vjp_de(const InstParams& ip, double nu, int n, int lo, int hi, const double* U, double* lam,
                              const double* gface_lo, const double* gface_hi) {
  Prim P[kMaxPencil];
  double dl[kMaxPencil][5], fa[kMaxPencil][5], fl[kMaxPencil];
  Par pa[kMaxPencil][5];
  double WL[kMaxPencil][5], WR[kMaxPencil][5];
  const double sixth = ip.sixth;
  for (int j = 0; j < n; j++) {
    double u6[6] = {U[j], U[n + j], U[2 * n + j], U[3 * n + j], U[4 * n + j], U[5 * n + j]};
    P[j] = prim_fwd_de(ip, u6);
  }
  for (int j = 1; j <= n - 2; j++)
    for (int v = 0; v < 5; v++) dl[j][v] = mc_slope(P[j - 1].q[v], P[j].q[v], P[j + 1].q[v]);
  for (int j = 1; j <= n - 3; j++)
    for (int v = 0; v < 5; v++)
      fa[j][v] = 0.5 * (P[j].q[v] + P[j + 1].q[v]) - (dl[j + 1][v] - dl[j][v]) * sixth;
  bool shk[kMaxPencil], fact[kMaxPencil];
  double rr_[kMaxPencil];
  for (int j = 2; j <= n - 3; j++) {
    const double pp1 = P[j + 1].q[4], pm1 = P[j - 1].q[4];
    const double dp1 = pp1 - pm1;
    const double pmin = pp1 < pm1 ? pp1 : pm1;
    shk[j] = (fabs(dp1) > 0.33 * pmin) && (P[j - 1].q[1] - P[j + 1].q[1] > 0.0);
    const double dp2 = P[j + 2].q[4] - P[j - 2].q[4];
    const double r = (dp2 != 0.0) ? dp1 / dp2 : 0.0;
    rr_[j] = r;
    double ft = 10.0 * (r - 0.75);
    fact[j] = shk[j] && dp2 != 0.0 && ft < 1.0 && ft > 0.0;
    ft = ft < 1.0 ? ft : 1.0;
    ft = ft > 0.0 ? ft : 0.0;
    fl[j] = shk[j] ? ft : 0.0;
    for (int v = 0; v < 5; v++) pa[j][v] = parabola(P[j].q[v], fa[j - 1][v], fa[j][v], fl[j], sixth);
    trace(ip, P[j].q[0], P[j].q[1], P[j].c, P[j].ir, pa[j], nu, WL[j], WR[j]);
  }
  // adjoint accumulators
  double gq[kMaxPencil][5] = {}, gc[kMaxPencil] = {}, gir[kMaxPencil] = {};
  double gdl[kMaxPencil][5] = {}, gfa[kMaxPencil][5] = {}, gfl[kMaxPencil] = {};
  double gWL[kMaxPencil][5] = {}, gWR[kMaxPencil][5] = {};
  // fluxes and Godunov velocities at the faces j+1/2, j = lo-1 .. hi-1
  double F[kMaxPencil][6], ugf[kMaxPencil], gug[kMaxPencil] = {};
  for (int j = lo - 1; j <= hi - 1; j++) riemann_flux<true>(ip, WL[j], WR[j + 1], F[j], &ugf[j]);
  // update U_j -= nu (F_{j+1/2} - F_{j-1/2}) on [lo, hi), rho e also less the
  // work nu p_j (u_g(j+1/2) - u_g(j-1/2)), then floors and resynchronisation:
  // the adjoint of the pre-floor values replaces lam there
  for (int j = lo; j < hi; j++) {
    double V[6], g[6];
    for (int v = 0; v < 6; v++) {
      V[v] = U[v * n + j] - nu * (F[j][v] - F[j - 1][v]);
      g[v] = lam[v * n + j];
    }
    V[5] = V[5] - nu * (P[j].q[4] * (ugf[j] - ugf[j - 1]));
    floor_vjp_de(ip, V, g, g);
    for (int v = 0; v < 6; v++) lam[v * n + j] = g[v];
    const double gw = -nu * g[5];
    gq[j][4] += gw * (ugf[j] - ugf[j - 1]);
    gug[j] += gw * P[j].q[4];
    gug[j - 1] -= gw * P[j].q[4];
  }
  // faces for reflux
  for (int j = lo - 1; j <= hi - 1; j++) {
    double gF[6];
    for (int v = 0; v < 6; v++) {
      const double up = (j + 1 >= lo && j + 1 < hi) ? lam[v * n + j + 1] : 0.0;
      const double dn = (j >= lo && j < hi) ? lam[v * n + j] : 0.0;
      gF[v] = nu * (up - dn);
    }
    if (j == lo - 1 && gface_lo)
      for (int v = 0; v < 6; v++) gF[v] += gface_lo[v];
    if (j == hi - 1 && gface_hi)
      for (int v = 0; v < 6; v++) gF[v] += gface_hi[v];
    riemann_vjp_n<64, true, true>(ip, WL[j], WR[j + 1], gF, gWL[j], gWR[j + 1], gF[5], gug[j]);
  }
  for (int j = 2; j <= n - 3; j++) {
    ParGrad G[5] = {};
    double grho = 0, gu = 0;
    trace_vjp(ip, P[j].q[0], P[j].q[1], P[j].c, P[j].ir, pa[j], nu, gWL[j], gWR[j], G, &grho, &gu, &gc[j], &gir[j]);
    gq[j][0] += grho;
    gq[j][1] += gu;
    for (int v = 0; v < 5; v++)
      parabola_vjp(P[j].q[v], fa[j - 1][v], fa[j][v], fl[j], sixth, G[v], &gq[j][v], &gfa[j - 1][v], &gfa[j][v],
                   &gfl[j]);
    if (fact[j]) {
      const double gr = 10.0 * gfl[j];
      const double dp2 = P[j + 2].q[4] - P[j - 2].q[4];
      const double gdp1 = gr / dp2, gdp2 = -gr * rr_[j] / dp2;
      gq[j + 1][4] += gdp1;
      gq[j - 1][4] -= gdp1;
      gq[j + 2][4] += gdp2;
      gq[j - 2][4] -= gdp2;
    }
  }
  for (int j = 1; j <= n - 3; j++)
    for (int v = 0; v < 5; v++) {
      const double g = gfa[j][v];
      gq[j][v] += 0.5 * g;
      gq[j + 1][v] += 0.5 * g;
      gdl[j + 1][v] -= sixth * g;
      gdl[j][v] += sixth * g;
    }
  for (int j = 1; j <= n - 2; j++)
    for (int v = 0; v < 5; v++)
      slope_vjp(P[j - 1].q[v], P[j].q[v], P[j + 1].q[v], gdl[j][v], &gq[j - 1][v], &gq[j][v], &gq[j + 1][v]);
  for (int j = 0; j < n; j++) {
    double u6[6] = {U[j], U[n + j], U[2 * n + j], U[3 * n + j], U[4 * n + j], U[5 * n + j]};
    double gU[6] = {0, 0, 0, 0, 0, 0};
    prim_vjp<true>(ip, u6, P[j], gq[j], gc[j], gir[j], gU);
    for (int v = 0; v < 6; v++) lam[v * n + j] += gU[v];
  }
}

}  // namespace amr
