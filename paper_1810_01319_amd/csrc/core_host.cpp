// core_host.cpp -- host build of the sweep formulas (ppm_core.hpp) and their
// adjoint (ppm_adjoint.hpp) for CPU unit tests of the adjoint against finite
// differences.  Not used by the GPU path.
#include <cstdint>
#include <cstring>

#include "ppm_adjoint.hpp"

using namespace amr;

static InstParams params(const double* gas, int iters) {
  InstParams p{};
  p.gamma = gas[0];
  p.gm1 = gas[0] - 1.0;
  p.inv_gm1 = 1.0 / (gas[0] - 1.0);
  p.g_gm1 = gas[0] / (gas[0] - 1.0);
  p.g1 = (gas[0] + 1.0) / (2.0 * gas[0]);
  p.rho_floor = gas[1];
  p.p_floor = gas[2];
  p.sixth = 1.0 / 6.0;
  p.two3 = 2.0 / 3.0;
  p.iters = iters;
  return p;
}

// gas = (gamma, rho_floor, p_floor, eta1, eta2) for the dual-energy calls
static InstParams params_de(const double* gas, int iters) {
  InstParams p = params(gas, iters);
  p.eta1 = gas[3];
  p.eta2 = gas[4];
  return p;
}

extern "C" {

// Forward update of one pencil (cells [lo,hi) updated, then floored);
// faces_out[10]: the fluxes at lo-1/2 and hi-1/2.
void core_pencil_update(const double* gas, int iters, double nu, int n, int lo, int hi, const double* U,
                        double* Uout, double* faces_out) {
  const InstParams ip = params(gas, iters);
  Prim P[kMaxPencil];
  double dl[kMaxPencil][5], fa[kMaxPencil][5], WL[kMaxPencil][5], WR[kMaxPencil][5], F[kMaxPencil][5];
  for (int j = 0; j < n; j++) {
    double u5[5] = {U[j], U[n + j], U[2 * n + j], U[3 * n + j], U[4 * n + j]};
    P[j] = prim_fwd(ip, u5);
  }
  for (int j = 1; j <= n - 2; j++)
    for (int v = 0; v < 5; v++) dl[j][v] = mc_slope(P[j - 1].q[v], P[j].q[v], P[j + 1].q[v]);
  for (int j = 1; j <= n - 3; j++)
    for (int v = 0; v < 5; v++)
      fa[j][v] = 0.5 * (P[j].q[v] + P[j + 1].q[v]) - (dl[j + 1][v] - dl[j][v]) * ip.sixth;
  for (int j = 2; j <= n - 3; j++) {
    const double pp1 = P[j + 1].q[4], pm1 = P[j - 1].q[4];
    const double dp1 = pp1 - pm1;
    const double pmin = pp1 < pm1 ? pp1 : pm1;
    const bool shock = (fabs(dp1) > 0.33 * pmin) && (P[j - 1].q[1] - P[j + 1].q[1] > 0.0);
    const double dp2 = P[j + 2].q[4] - P[j - 2].q[4];
    const double r = (dp2 != 0.0) ? dp1 / dp2 : 0.0;
    double ft = 10.0 * (r - 0.75);
    ft = ft < 1.0 ? ft : 1.0;
    ft = ft > 0.0 ? ft : 0.0;
    const double f = shock ? ft : 0.0;
    Par pa[5];
    for (int v = 0; v < 5; v++) pa[v] = parabola(P[j].q[v], fa[j - 1][v], fa[j][v], f, ip.sixth);
    trace(ip, P[j].q[0], P[j].q[1], P[j].c, P[j].ir, pa, nu, WL[j], WR[j]);
  }
  for (int j = lo - 1; j <= hi - 1; j++) riemann_flux(ip, WL[j], WR[j + 1], F[j]);
  std::memcpy(Uout, U, sizeof(double) * 5 * n);
  for (int j = lo; j < hi; j++) {
    double V[5], W[5];
    for (int v = 0; v < 5; v++) V[v] = U[v * n + j] - nu * (F[j][v] - F[j - 1][v]);
    floor_apply(ip, V, W);
    for (int v = 0; v < 5; v++) Uout[v * n + j] = W[v];
  }
  for (int v = 0; v < 5; v++) {
    faces_out[v] = F[lo - 1][v];
    faces_out[5 + v] = F[hi - 1][v];
  }
}

// Dual energy: the same update with the sixth field rho e (U, Uout: six
// fields; faces_out[12]).
void core_pencil_update_de(const double* gas, int iters, double nu, int n, int lo, int hi, const double* U,
                           double* Uout, double* faces_out) {
  const InstParams ip = params_de(gas, iters);
  Prim P[kMaxPencil];
  double dl[kMaxPencil][5], fa[kMaxPencil][5], WL[kMaxPencil][5], WR[kMaxPencil][5], F[kMaxPencil][6],
      ug[kMaxPencil];
  for (int j = 0; j < n; j++) {
    double u6[6] = {U[j], U[n + j], U[2 * n + j], U[3 * n + j], U[4 * n + j], U[5 * n + j]};
    P[j] = prim_fwd_de(ip, u6);
  }
  for (int j = 1; j <= n - 2; j++)
    for (int v = 0; v < 5; v++) dl[j][v] = mc_slope(P[j - 1].q[v], P[j].q[v], P[j + 1].q[v]);
  for (int j = 1; j <= n - 3; j++)
    for (int v = 0; v < 5; v++)
      fa[j][v] = 0.5 * (P[j].q[v] + P[j + 1].q[v]) - (dl[j + 1][v] - dl[j][v]) * ip.sixth;
  for (int j = 2; j <= n - 3; j++) {
    const double pp1 = P[j + 1].q[4], pm1 = P[j - 1].q[4];
    const double dp1 = pp1 - pm1;
    const double pmin = pp1 < pm1 ? pp1 : pm1;
    const bool shock = (fabs(dp1) > 0.33 * pmin) && (P[j - 1].q[1] - P[j + 1].q[1] > 0.0);
    const double dp2 = P[j + 2].q[4] - P[j - 2].q[4];
    const double r = (dp2 != 0.0) ? dp1 / dp2 : 0.0;
    double ft = 10.0 * (r - 0.75);
    ft = ft < 1.0 ? ft : 1.0;
    ft = ft > 0.0 ? ft : 0.0;
    const double f = shock ? ft : 0.0;
    Par pa[5];
    for (int v = 0; v < 5; v++) pa[v] = parabola(P[j].q[v], fa[j - 1][v], fa[j][v], f, ip.sixth);
    trace(ip, P[j].q[0], P[j].q[1], P[j].c, P[j].ir, pa, nu, WL[j], WR[j]);
  }
  for (int j = lo - 1; j <= hi - 1; j++) riemann_flux<true>(ip, WL[j], WR[j + 1], F[j], &ug[j]);
  std::memcpy(Uout, U, sizeof(double) * 6 * n);
  for (int j = lo; j < hi; j++) {
    double V[6], W[6];
    for (int v = 0; v < 6; v++) V[v] = U[v * n + j] - nu * (F[j][v] - F[j - 1][v]);
    V[5] = V[5] - nu * (P[j].q[4] * (ug[j] - ug[j - 1]));
    floor_apply_de(ip, V, W);
    for (int v = 0; v < 6; v++) Uout[v * n + j] = W[v];
  }
  for (int v = 0; v < 6; v++) {
    faces_out[v] = F[lo - 1][v];
    faces_out[6 + v] = F[hi - 1][v];
  }
}

void core_pencil_vjp_de(const double* gas, int iters, double nu, int n, int lo, int hi, const double* U,
                        double* lam, const double* gface /* 12 or null */) {
  const InstParams ip = params_de(gas, iters);
  pencil_vjp_de(ip, nu, n, lo, hi, U, lam, gface, gface ? gface + 6 : nullptr);
}

void core_floor_de(const double* gas, const double* V, double* out) {
  const InstParams ip = params_de(gas, 5);
  floor_apply_de(ip, V, out);
}

void core_floor_vjp_de(const double* gas, const double* V, const double* g, double* gV) {
  const InstParams ip = params_de(gas, 5);
  floor_vjp_de(ip, V, g, gV);
}

void core_pencil_vjp(const double* gas, int iters, double nu, int n, int lo, int hi, const double* U, double* lam,
                     const double* gface /* 10 or null */) {
  const InstParams ip = params(gas, iters);
  pencil_vjp(ip, nu, n, lo, hi, U, lam, gface, gface ? gface + 5 : nullptr);
}

// post-update floors of one cell (pencil roles) and their adjoint
void core_floor(const double* gas, const double* V, double* out) {
  const InstParams ip = params(gas, 5);
  floor_apply(ip, V, out);
}

void core_floor_vjp(const double* gas, const double* V, const double* g, double* gV) {
  const InstParams ip = params(gas, 5);
  floor_vjp(ip, V, g, gV);
}

void core_riemann(const double* gas, int iters, const double* L, const double* R, double* F) {
  const InstParams ip = params(gas, iters);
  riemann_flux(ip, L, R, F);
}

void core_riemann_vjp(const double* gas, int iters, const double* L, const double* R, const double* gF, double* gL,
                      double* gR) {
  const InstParams ip = params(gas, iters);
  for (int v = 0; v < 5; v++) gL[v] = gR[v] = 0.0;
  riemann_vjp(ip, L, R, gF, gL, gR);
}

// the same transpose with every Newton evaluation reversed one by one
void core_riemann_vjp_stepwise(const double* gas, int iters, const double* L, const double* R, const double* gF,
                               double* gL, double* gR) {
  const InstParams ip = params(gas, iters);
  for (int v = 0; v < 5; v++) gL[v] = gR[v] = 0.0;
  riemann_vjp_n<64, false>(ip, L, R, gF, gL, gR);
}

}  // extern "C"

extern "C" {

// trace of one cell from its primitives q (rho,u,v,w,p), c, 1/rho and the 5
// parabolas (qL, qR, dq, q6 each): WL, WR
void core_trace(const double* gas, double rho, double u, double c, double ir, const double* par, double nu,
                double* WL, double* WR) {
  const InstParams ip = params(gas, 5);
  Par pa[5];
  for (int v = 0; v < 5; v++) pa[v] = Par{par[4 * v], par[4 * v + 1], par[4 * v + 2], par[4 * v + 3]};
  trace(ip, rho, u, c, ir, pa, nu, WL, WR);
}

// out: g of par (20), then grho, gu, gc, gir
void core_trace_vjp(const double* gas, double rho, double u, double c, double ir, const double* par, double nu,
                    const double* gWL, const double* gWR, double* out) {
  const InstParams ip = params(gas, 5);
  Par pa[5];
  for (int v = 0; v < 5; v++) pa[v] = Par{par[4 * v], par[4 * v + 1], par[4 * v + 2], par[4 * v + 3]};
  ParGrad G[5] = {};
  double grho = 0, gu = 0, gc = 0, gir = 0;
  trace_vjp(ip, rho, u, c, ir, pa, nu, gWL, gWR, G, &grho, &gu, &gc, &gir);
  for (int v = 0; v < 5; v++) {
    out[4 * v] = G[v].qL;
    out[4 * v + 1] = G[v].qR;
    out[4 * v + 2] = G[v].dq;
    out[4 * v + 3] = G[v].q6;
  }
  out[20] = grho;
  out[21] = gu;
  out[22] = gc;
  out[23] = gir;
}

// parabola of one field: out (qL, qR, dq, q6)
void core_parabola(double q, double qL, double qR, double f, double* out) {
  Par P = parabola(q, qL, qR, f, 1.0 / 6.0);
  out[0] = P.qL; out[1] = P.qR; out[2] = P.dq; out[3] = P.q6;
}

// g of (qL, qR, dq, q6) -> out (gq, gqL, gqR, gf)
void core_parabola_vjp(double q, double qL, double qR, double f, const double* g, double* out) {
  ParGrad G{g[0], g[1], g[2], g[3]};
  out[0] = out[1] = out[2] = out[3] = 0.0;
  parabola_vjp(q, qL, qR, f, 1.0 / 6.0, G, &out[0], &out[1], &out[2], &out[3]);
}

}  // extern "C"
