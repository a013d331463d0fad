// adjoint.hip -- kernels of the hand-written adjoint of one hydro step:
// transposes of reflux, of the three sweeps (recomputed from their stored
// inputs, branches taken from the forward) and of the ghost refresh.
//
// The adjoint of the step U_out = Reflux(Sweep3(Sweep2(Sweep1(Refresh(U_in)))))
// with dt frozen is applied to lam in place: lam enters as dL/dU_out and
// leaves as dL/dU_in.  Ghost entries of lam are zero on entry and on exit
// (ghost values of a state are overwritten by the next refresh).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "adjoint.hpp"
#include "ghost.hpp"
#include "xcd.hpp"
#include "ppm_adjoint.hpp"

namespace amr {
namespace {

constexpr int G = kGhost;

__device__ __forceinline__ double level_dx_a(const InstParams& ip, int N, int l) {
  return 1.0 / (double)((int64_t)ip.root[0] * N << l);
}

__global__ void fill_zero(double* __restrict__ p, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0.0;
}

// Reflux transpose: each coarse face cell's correction
// U_c += s nu_c (F_c - ((F00 + F10) + (F01 + F11)) / 4) sends s nu_c lam_c to
// the coarse face flux and -s nu_c lam_c / 4 to each of its four fine fluxes.
template <int N, int DIR, int NF>
__global__ void __launch_bounds__(256) reflux_adjoint(const double* __restrict__ lam, const double* __restrict__ dtv,
                                                      DevPlan P, double* __restrict__ gfaces) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int A = DIR == 0 ? 1 : 0;
  constexpr int B = DIR == 2 ? 1 : 2;
  constexpr int SD = DIR == 0 ? 1 : (DIR == 1 ? M : M * M);
  constexpr int SA = A == 0 ? 1 : (A == 1 ? M : M * M);
  constexpr int SB = B == 0 ? 1 : (B == 1 ? M : M * M);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nreflux[DIR] * N * N) return;
  const int k = int(t / (N * N));
  const int r = int(t - int64_t(k) * N * N);
  const int tA = r % N, tB = r / N;
  const RefluxTask T = P.reflux[DIR][k];
  const BlockInfo bi = P.blocks[T.leaf];
  const InstParams& ip = P.inst[bi.inst];
  const double nu = dtv[bi.inst] / level_dx_a(ip, N, bi.level);
  const int hA = tA >= N / 2, hB = tB >= N / 2;
  const int fs = T.slot_f[hA + 2 * hB];
  const int fA = 2 * tA - hA * N, fB = 2 * tB - hB * N;
  const int d = T.side ? N + G - 1 : G;
  const double* cellp = lam + int64_t(T.leaf) * NF * M3 + int64_t(d) * SD + int64_t(G + tA) * SA +
                        int64_t(G + tB) * SB;
  const double s = T.side ? 1.0 : -1.0;
#pragma unroll
  for (int f = 0; f < NF; f++) {
    const double g = s * nu * cellp[f * M3];
    gfaces[(int64_t(T.slot_c) * NF + f) * N * N + int64_t(tB) * N + tA] = g;
    double* Q = gfaces + (int64_t(fs) * NF + f) * N * N;
    const double gf = -0.25 * g;
    Q[fB * N + fA] = gf;
    Q[fB * N + fA + 1] = gf;
    Q[(fB + 1) * N + fA] = gf;
    Q[(fB + 1) * N + fA + 1] = gf;
  }
}

// Sweep transpose, LDS-staged: a workgroup holds R whole pencils, one thread
// per cell.  The forward sweep is recomputed phase by phase (primitives,
// slopes, face values, flattening + parabolas + tracing, Riemann fluxes) and
// its intermediates kept in LDS; the reverse phases then run in the opposite
// order, each cell gathering what its neighbours' products send it, so no
// two threads ever add to the same entry.
// Tile shape per block size and axis (measured on gfx950: x sweeps, whose
// tiles are contiguous rows, run best with smaller tiles; y and z best with
// 6 pencils, 4 waves per workgroup).
template <int N, int DIR>
struct AdjShape {
  static constexpr int M = N + 2 * G;
  static constexpr int R = N == 8 ? 9 : (N == 16 ? 11 : (DIR == 0 ? 3 : 6));  // pencils per tile
  static constexpr int T = R * M;                                              // cells per tile
  static constexpr int WG = ((T + 63) / 64) * 64;
};

// FLOORS: the variant with the post-update floors' products (and the flux
// recompute that detects them).  When the host knows the forward step's
// floor-reset count (sel >= 0: whether it is non-zero) only the matching
// variant is launched; otherwise both are, and each returns at once unless
// the count on the device (null: unknown, the floors variant) selects it.
// Registers are capped for 3 waves per SIMD (a few bytes of spill cost less
// than the lost occupancy).  The cell's state and adjoint are read together
// at the start (the adjoint parked in LDS until the reverse pass) and again
// one phase before the end, so that their latency overlaps computation.
template <int N, int DIR, bool FLOORS, int NF = kFields>
__global__ void __launch_bounds__((AdjShape<N, DIR>::WG)) __attribute__((amdgpu_waves_per_eu(3)))
sweep_adjoint(const double* __restrict__ Uin, double* __restrict__ lam, const double* __restrict__ dtv, DevPlan P,
              const double* __restrict__ gfaces, const unsigned long long* __restrict__ floors, int sel, int loA,
              int nA, int loB, int nB) {
  using S = AdjShape<N, DIR>;
  constexpr int M = S::M, R = S::R, T = S::T;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int A = DIR == 0 ? 1 : 0;
  constexpr int B = DIR == 2 ? 1 : 2;
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
  constexpr int SD = DIR == 0 ? 1 : (DIR == 1 ? M : M * M);
  constexpr int SA = A == 0 ? 1 : (A == 1 ? M : M * M);
  constexpr int SB = B == 0 ? 1 : (B == 1 ? M : M * M);
  constexpr int NS = DIR == 0 ? 1 : R;  // item stride between neighbouring cells
  constexpr bool DE = NF == kFieldsDE;  // dual-energy field rho e (field 5); only with FLOORS
  static_assert(!DE || FLOORS, "the dual-energy transpose recomputes the fluxes");
  constexpr int fmap[6] = {0, 1 + DIR, 1 + T1, 1 + T2, 4, 5};
  __shared__ double Ps[5][T];  // primitives
  __shared__ double Xs[5][T];  // slopes; fluxes; adjoint sent to face c-1/2
  __shared__ double Ys[5][T];  // face values at c+1/2; adjoint sent to cell c-1
  __shared__ double Ws[5][T];  // right states at c-1/2 and their adjoint; adjoint sent to cell c+1
  __shared__ double Ls[NF][T];  // adjoint of the pre-floor update; adjoint sent to face c+1/2
  __shared__ double Fl[2][T];  // flattening adjoint sent to p of cells c+-1, c+-2
  __shared__ double Gs[DE ? 2 : 1][DE ? T : 1];  // DE: rho e flux and Godunov velocity at c+1/2
  // a tile is R consecutive pencils of the leaf's nA x nB plane (numbered
  // along A, then B), so only the leaf's last tile is partial
  const int npen = nA * nB;
  const int tpl = (npen + R - 1) / R;
  const unsigned bx = xcd_block();
  const int s = int(bx / unsigned(tpl));
  const int i = threadIdx.x;
  const int r = DIR == 0 ? i / M : i % R;
  const int c = DIR == 0 ? i - r * M : i / R;
  const int pp = (int(bx) - s * tpl) * R + r;
  const bool live = i < T && pp < npen;
  const int iB = loB + pp / nA;
  const BlockInfo bi = P.blocks[s];
  const InstParams ip = P.inst[bi.inst];  // by value: read once, before any store
  const double nu = dtv[bi.inst] / level_dx_a(ip, N, bi.level);
  const int iA = loA + pp % nA;
  const int64_t off = int64_t(s) * NF * M3 + int64_t(iA) * SA + int64_t(iB) * SB + int64_t(c) * SD;
  const double* const ucell = Uin + off;
  double* const lcell = lam + off;
  const double sixth = ip.sixth;
  const bool traced = live && c >= 2 && c <= M - 3;
  const bool faced = live && c >= 2 && c <= M - 4;
  const bool active = live && c >= G && c < G + N;
  // sel < 0: the device count selects (uniform over the grid); else the host's choice
  const bool with_floors = sel < 0 ? (floors == nullptr || *floors != 0) : sel != 0;
  if (with_floors != FLOORS) return;

  // ---- forward recompute ----
  // Between phases only adjoint accumulators stay in registers: primitives
  // are read back from Ps, c and 1/rho wait in Fl until the trace adjoint,
  // the flattening is recomputed where needed, and the floor-free variant
  // keeps the left states in Xs (free between the face values and the trace
  // adjoint).
  if (live) {
    // the cell's adjoint is read with its state (one memory round trip) and
    // waits in Ls, which the forward recompute does not use
    double u5[NF], l5[NF];
#pragma unroll
    for (int v = 0; v < NF; v++) {
      u5[v] = ucell[fmap[v] * M3];
      l5[v] = lcell[fmap[v] * M3];
    }
    Prim Pr;
    if constexpr (DE) Pr = prim_fwd_de(ip, u5);
    else Pr = prim_fwd(ip, u5);
#pragma unroll
    for (int v = 0; v < 5; v++) Ps[v][i] = Pr.q[v];
#pragma unroll
    for (int v = 0; v < NF; v++) Ls[v][i] = l5[v];
    Fl[0][i] = Pr.c;
    Fl[1][i] = Pr.ir;
  }
  __syncthreads();
  if (live && c >= 1 && c <= M - 2) {
#pragma unroll
    for (int v = 0; v < 5; v++) Xs[v][i] = mc_slope(Ps[v][i - NS], Ps[v][i], Ps[v][i + NS]);
  }
  __syncthreads();
  if (live && c >= 1 && c <= M - 3) {
#pragma unroll
    for (int v = 0; v < 5; v++)
      Ys[v][i] = 0.5 * (Ps[v][i] + Ps[v][i + NS]) - (Xs[v][i + NS] - Xs[v][i]) * sixth;
  }
  __syncthreads();
  // flattening of the own cell: coefficient f, whether it is interior to its
  // clamps (fact), the pressure-jump ratio and its denominator
  auto flattening = [&](double& f, double& rr, double& dp2, bool& fact) {
    const double pp1 = Ps[4][i + NS], pm1 = Ps[4][i - NS];
    const double dp1 = pp1 - pm1;
    const double pmin = pp1 < pm1 ? pp1 : pm1;
    const bool shock = (fabs(dp1) > 0.33 * pmin) && (Ps[1][i - NS] - Ps[1][i + NS] > 0.0);
    dp2 = Ps[4][i + 2 * NS] - Ps[4][i - 2 * NS];
    rr = (dp2 != 0.0) ? dp1 / dp2 : 0.0;
    double ft = 10.0 * (rr - 0.75);
    fact = shock && dp2 != 0.0 && ft < 1.0 && ft > 0.0;
    ft = ft < 1.0 ? ft : 1.0;
    ft = ft > 0.0 ? ft : 0.0;
    f = shock ? ft : 0.0;
  };
  double WL[5] = {0, 0, 0, 0, 0};  // held in registers by the floor variant only
  if (traced) {
    double f, rr, dp2;
    bool fact;
    flattening(f, rr, dp2, fact);
    Par pa[5];
#pragma unroll
    for (int v = 0; v < 5; v++) pa[v] = parabola(Ps[v][i], Ys[v][i - NS], Ys[v][i], f, sixth);
    double WR[5];
    trace(ip, Ps[0][i], Ps[1][i], Fl[0][i], Fl[1][i], pa, nu, WL, WR);
#pragma unroll
    for (int v = 0; v < 5; v++) {
      Ws[v][i] = WR[v];
      if (!FLOORS) Xs[v][i] = WL[v];
    }
  }
  __syncthreads();
  if (FLOORS) {
    if (faced) {
      double R5[5], F[NF], ug = 0.0;
#pragma unroll
      for (int v = 0; v < 5; v++) R5[v] = Ws[v][i + NS];
      riemann_flux<DE>(ip, WL, R5, F, &ug);
#pragma unroll
      for (int v = 0; v < 5; v++) Xs[v][i] = F[v];
      if constexpr (DE) {
        Gs[0][i] = F[5];
        Gs[1][i] = ug;
      }
    }
    __syncthreads();
  }

  // ---- reverse ----
  // update and floors: li is the adjoint of the cell's own input through the
  // identity part (pre-floor adjoint on active cells, unchanged elsewhere);
  // the floor-free variant rereads it from lam at the end
  double li[NF] = {};
  if (live) {
    if (FLOORS) {
#pragma unroll
      for (int v = 0; v < NF; v++) li[v] = Ls[v][i];
      if (active) {
        double V[NF];
#pragma unroll
        for (int v = 0; v < 5; v++) V[v] = ucell[fmap[v] * M3] - nu * (Xs[v][i] - Xs[v][i - NS]);
        if constexpr (DE) {
          // rho e: its flux difference, then the work of the cell's pressure
          V[5] = ucell[fmap[5] * M3] - nu * (Gs[0][i] - Gs[0][i - NS]);
          V[5] = V[5] - nu * (Ps[4][i] * (Gs[1][i] - Gs[1][i - NS]));
          floor_vjp_de(ip, V, li, li);
        } else {
          floor_vjp(ip, V, li, li);
        }
      }
#pragma unroll
      for (int v = 0; v < NF; v++) Ls[v][i] = active ? li[v] : 0.0;
    } else if (!active) {
#pragma unroll
      for (int v = 0; v < 5; v++) Ls[v][i] = 0.0;
    }
  }
  __syncthreads();
  // Riemann flux at c+1/2: adjoint of the left state (own) and of the right
  // state (cell c+1, through Ws)
  double gWL[5] = {0, 0, 0, 0, 0};
  if (faced) {
    double gF[5], L5[5], R5[5], gR5[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 5; v++) {
      gF[v] = nu * (Ls[v][i + NS] - Ls[v][i]);
      L5[v] = FLOORS ? WL[v] : Xs[v][i];
      R5[v] = Ws[v][i + NS];
    }
    const bool faces_act = iA >= G && iA < G + N && iB >= G && iB < G + N;
    double gF5 = 0.0, gug = 0.0;
    if constexpr (DE) {
      // rho e's flux, and the Godunov velocity through the work terms of the
      // cells c (-nu p_c) and c+1 (+nu p_c+1)
      gF5 = nu * (Ls[5][i + NS] - Ls[5][i]);
      gug = nu * (Ps[4][i + NS] * Ls[5][i + NS] - Ps[4][i] * Ls[5][i]);
    }
    if (faces_act && (c == G - 1 || c == N + G - 1)) {
      const int slot = P.faceslot[6 * int64_t(s) + 2 * DIR + (c == G - 1 ? 0 : 1)];
      if (slot >= 0) {
        const double* gf = gfaces + int64_t(slot) * NF * N * N + int64_t(iB - G) * N + (iA - G);
#pragma unroll
        for (int v = 0; v < 5; v++) gF[v] += gf[fmap[v] * N * N];
        if constexpr (DE) gF5 += gf[5 * N * N];
      }
    }
    riemann_vjp_n<kAdjMaxIters, true, DE>(ip, L5, R5, gF, gWL, gR5, gF5, gug);
#pragma unroll
    for (int v = 0; v < 5; v++) Ws[v][i + NS] = gR5[v];
  }
  __syncthreads();
  // tracing, parabolas and flattening of the own cell; the adjoints sent to
  // the faces c-1/2 and c+1/2 go to Xs and Ls field by field
  double gq[5] = {0, 0, 0, 0, 0}, gc = 0, gir = 0;
  if (live) {
    double gd1 = 0, gd2 = 0;
    if (traced) {
      double f;
      {
        double rr, dp2;
        bool fact;
        flattening(f, rr, dp2, fact);
      }
      const double cs = Fl[0][i], ir = Fl[1][i];
      double gfl = 0;
      // transverse fields, one at a time
#pragma unroll
      for (int v = 2; v <= 3; v++) {
        const double qv = Ps[v][i], fL = Ys[v][i - NS], fR = Ys[v][i];
        const Par pv = parabola(qv, fL, fR, f, sixth);
        ParGrad Gv = {0, 0, 0, 0};
        trace_vjp_transverse(Ps[1][i], nu, ip.two3, pv, gWL[v], c >= 3 ? Ws[v][i] : 0.0, &Gv, &gq[1]);
        double glo = 0, ghi = 0;
        parabola_vjp(qv, fL, fR, f, sixth, Gv, &gq[v], &glo, &ghi, &gfl);
        Xs[v][i] = glo;
        Ls[v][i] = ghi;
      }
      // rho, u, p
      constexpr int cf[3] = {0, 1, 4};
      double gWR[5];
#pragma unroll
      for (int v = 0; v < 5; v++) gWR[v] = c >= 3 ? Ws[v][i] : 0.0;
      Par pc[3];
#pragma unroll
      for (int k = 0; k < 3; k++) pc[k] = parabola(Ps[cf[k]][i], Ys[cf[k]][i - NS], Ys[cf[k]][i], f, sixth);
      ParGrad Gc[3] = {};
      double grho = 0, gu = 0;
      trace_vjp_rup(ip, Ps[0][i], Ps[1][i], cs, ir, pc[0], pc[1], pc[2], nu, gWL, gWR, &Gc[0], &Gc[1], &Gc[2],
                    &grho, &gu, &gc, &gir);
      gq[0] += grho;
      gq[1] += gu;
#pragma unroll
      for (int k = 0; k < 3; k++) {
        double glo = 0, ghi = 0;
        parabola_vjp(Ps[cf[k]][i], Ys[cf[k]][i - NS], Ys[cf[k]][i], f, sixth, Gc[k], &gq[cf[k]], &glo, &ghi, &gfl);
        Xs[cf[k]][i] = glo;
        Ls[cf[k]][i] = ghi;
      }
      double f2, rr, dp2;  // recomputed here rather than held across the trace adjoint
      bool fact;
      flattening(f2, rr, dp2, fact);
      if (fact) {
        const double gr = 10.0 * gfl;
        gd1 = gr / dp2;
        gd2 = -gr * rr / dp2;
      }
    } else {
#pragma unroll
      for (int v = 0; v < 5; v++) {
        Xs[v][i] = 0.0;
        Ls[v][i] = 0.0;
      }
    }
    Fl[0][i] = gd1;
    Fl[1][i] = gd2;
  }
  __syncthreads();
  // face values at c+-1/2, flattening, then the own slope; the state and
  // (floor-free variant) the adjoint of the cell, needed at the end, are
  // read here so that the two phases hide their latency
  double u5e[NF] = {};
  if (live) {
#pragma unroll
    for (int v = 0; v < NF; v++) u5e[v] = ucell[fmap[v] * M3];
    if (!FLOORS) {
#pragma unroll
      for (int v = 0; v < 5; v++) li[v] = lcell[fmap[v] * M3];
    }
#pragma unroll
    for (int v = 0; v < 5; v++) {
      const double ghi = (c >= 1 && c <= M - 3) ? Ls[v][i] + Xs[v][i + NS] : 0.0;
      const double glo = (c >= 2 && c <= M - 2) ? Ls[v][i - NS] + Xs[v][i] : 0.0;
      gq[v] += 0.5 * (ghi + glo);
      double gm = 0, gp = 0;
      if (c >= 1 && c <= M - 2) {
        const double gdl = sixth * (ghi - glo);
        slope_vjp(Ps[v][i - NS], Ps[v][i], Ps[v][i + NS], gdl, &gm, &gq[v], &gp);
      }
      Ys[v][i] = gm;
      Ws[v][i] = gp;
    }
    double gp4 = 0;
    if (c >= 1) gp4 += Fl[0][i - NS];
    if (c + 1 < M) gp4 -= Fl[0][i + NS];
    if (c >= 2) gp4 += Fl[1][i - 2 * NS];
    if (c + 2 < M) gp4 -= Fl[1][i + 2 * NS];
    gq[4] += gp4;
  }
  __syncthreads();
  // neighbours' slopes, primitives, and the new adjoint of the cell
  if (live) {
#pragma unroll
    for (int v = 0; v < 5; v++) {
      if (c >= 1) gq[v] += Ws[v][i - NS];
      if (c + 1 < M) gq[v] += Ys[v][i + NS];
    }
    double gU[NF] = {};
    if constexpr (DE) {
      // the work term of the own update: -nu p (u_g(c+1/2) - u_g(c-1/2)) on rho e
      if (active) gq[4] += -nu * (Gs[1][i] - Gs[1][i - NS]) * li[5];
      const Prim Pr = prim_fwd_de(ip, u5e);
      prim_vjp<true>(ip, u5e, Pr, gq, gc, gir, gU);
    } else {
      const Prim Pr = prim_fwd(ip, u5e);
      prim_vjp(ip, u5e, Pr, gq, gc, gir, gU);
    }
#pragma unroll
    for (int v = 0; v < NF; v++) lcell[fmap[v] * M3] = li[v] + gU[v];
  }
}

// Refresh transpose, phase 2 (prolongation): a prolonged ghost's adjoint
// goes to the coarse parent cell and, through the frozen minmod slopes, to
// its face neighbours; then the ghost entry is cleared.
// One thread per ghost cell of every leaf with a coarser neighbour (the
// threads of other neighbours return at once: spreading the prolonged cells
// over the grid keeps fewer waves adding to one coarse cell at a time than
// the forward's compact task list would).
template <int N, int NF>
__global__ void __launch_bounds__(256) refresh2_adjoint(double* __restrict__ lam, const double* __restrict__ Uref,
                                                        DevPlan P) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int GC = M * M * M - N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.np2 * GC) return;
  const int w = int(t / GC);
  const int g = int(t - int64_t(w) * GC);
  const int s = P.p2list[w];
  int a, b, c;
  ghost_decode<N>(g, a, b, c);
  const Nbr e = P.nbr[27 * int64_t(s) + dir_code<N>(a, b, c)];
  if (e.kind != NBR_COARSE) return;
  const BlockInfo bi = P.blocks[s];
  const InstParams& ip = P.inst[bi.inst];
  const int l = bi.level;
  const int px = bc_index<N>(ip, l, 0, bi.i * N + a - G);
  const int py = bc_index<N>(ip, l, 1, bi.j * N + b - G);
  const int pz = bc_index<N>(ip, l, 2, bi.k * N + c - G);
  const BlockInfo cb = P.blocks[e.id];
  const int la = (px >> 1) - cb.i * N + G, lb = (py >> 1) - cb.j * N + G, lc = (pz >> 1) - cb.k * N + G;
  const double o[3] = {(px & 1) ? 0.25 : -0.25, (py & 1) ? 0.25 : -0.25, (pz & 1) ? 0.25 : -0.25};
  const int64_t cbase = int64_t(e.id) * NF * M3 + (int64_t(lc) * M + lb) * M + la;
  const int64_t gidx = int64_t(s) * NF * M3 + (int64_t(c) * M + b) * M + a;
  const int st[3] = {1, M, M * M};
#pragma unroll
  for (int f = 0; f < NF; f++) {
    double* lg = lam + gidx + f * M3;
    const double gv = *lg;
    *lg = 0.0;
    if (gv == 0.0) continue;
    const double* q = Uref + cbase + f * M3;
    const double u0 = q[0];
    double g0 = gv;
    for (int d = 0; d < 3; d++) {
      // s_d = minmod(q[+1] - u0, u0 - q[-1]); the branch the forward took
      const double aa = q[st[d]] - u0, bb = u0 - q[-st[d]];
      if (!(aa * bb > 0.0)) continue;
      const double gs = o[d] * gv;
      if (fabs(aa) < fabs(bb)) {
        atomicAdd(lam + cbase + f * M3 + st[d], gs);
        g0 -= gs;
      } else {
        g0 += gs;
        atomicAdd(lam + cbase + f * M3 - st[d], -gs);
      }
    }
    atomicAdd(lam + cbase + f * M3, g0);
  }
}

// Refresh transpose, phase 1 (copies and restriction): a ghost's adjoint goes
// to its source cell (weight 1) or to its 8 children (weight 1/8); then the
// ghost entry is cleared.
template <int N, int NF>
__global__ void __launch_bounds__(256) refresh1_adjoint(double* __restrict__ lam, DevPlan P) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int GC = M * M * M - N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * GC) return;
  const int s = int(t / GC);
  const int g = int(t - int64_t(s) * GC);
  int a, b, c;
  ghost_decode<N>(g, a, b, c);
  const Nbr e = P.nbr[27 * int64_t(s) + dir_code<N>(a, b, c)];
  if (e.kind == NBR_COARSE) return;
  const BlockInfo bi = P.blocks[s];
  const InstParams& ip = P.inst[bi.inst];
  const int l = bi.level;
  const int px = bc_index<N>(ip, l, 0, bi.i * N + a - G);
  const int py = bc_index<N>(ip, l, 1, bi.j * N + b - G);
  const int pz = bc_index<N>(ip, l, 2, bi.k * N + c - G);
  double* dst = lam + int64_t(s) * NF * M3 + (int64_t(c) * M + b) * M + a;
  if (e.kind == NBR_COPY) {
    const BlockInfo sb = P.blocks[e.id];
    const int la = px - sb.i * N + G, lb = py - sb.j * N + G, lc = pz - sb.k * N + G;
    double* src = lam + int64_t(e.id) * NF * M3 + (int64_t(lc) * M + lb) * M + la;
#pragma unroll
    for (int f = 0; f < NF; f++) {
      const double gv = dst[f * M3];
      dst[f * M3] = 0.0;
      if (gv != 0.0) atomicAdd(src + f * M3, gv);
    }
  } else {
    const int qx = 2 * px, qy = 2 * py, qz = 2 * pz;
    const int cidx = ((qx / N) & 1) + 2 * ((qy / N) & 1) + 4 * ((qz / N) & 1);
    const int fs = P.fine[8 * int64_t(e.id) + cidx];
    const int la = qx % N + G, lb = qy % N + G, lc = qz % N + G;
    double* src = lam + int64_t(fs) * NF * M3 + (int64_t(lc) * M + lb) * M + la;
#pragma unroll
    for (int f = 0; f < NF; f++) {
      const double gv = dst[f * M3];
      dst[f * M3] = 0.0;
      if (gv == 0.0) continue;
      const double g8 = gv * 0.125;
      double* q = src + f * M3;
      atomicAdd(q, g8);
      atomicAdd(q + 1, g8);
      atomicAdd(q + M, g8);
      atomicAdd(q + M + 1, g8);
      atomicAdd(q + M * M, g8);
      atomicAdd(q + M * M + 1, g8);
      atomicAdd(q + M * M + M, g8);
      atomicAdd(q + M * M + M + 1, g8);
    }
  }
}

inline unsigned gridn(int64_t n, int b) { return unsigned((n + b - 1) / b); }

template <int N, int DIR>
hipError_t sweep_adj_nd(const DevPlan& P, const double* Uin, double* lam, const double* dt, const double* gfaces,
                        const unsigned long long* floors, int64_t floors_host, const int swept[3], hipStream_t st) {
  using S = AdjShape<N, DIR>;
  constexpr int A = DIR == 0 ? 1 : 0, B = DIR == 2 ? 1 : 2;
  const int loA = swept[A] ? G : 0, nA = swept[A] ? N : S::M;
  const int loB = swept[B] ? G : 0, nB = swept[B] ? N : S::M;
  const int64_t tiles = P.nleaf * ((int64_t(nA) * nB + S::R - 1) / S::R);
  if (tiles == 0) return hipSuccess;
  const dim3 g(static_cast<unsigned>(tiles)), b(S::WG);
  if (P.nf == kFieldsDE) {  // one variant: the flux recompute the dual-energy transpose needs
    hipLaunchKernelGGL((sweep_adjoint<N, DIR, true, kFieldsDE>), g, b, 0, st, Uin, lam, dt, P, gfaces, floors, 1, loA,
                       nA, loB, nB);
    return hipGetLastError();
  }
  const int sel = floors == nullptr ? 1 : (floors_host < 0 ? -1 : (floors_host > 0 ? 1 : 0));
  if (sel <= 0)
    hipLaunchKernelGGL((sweep_adjoint<N, DIR, false>), g, b, 0, st, Uin, lam, dt, P, gfaces, floors, sel, loA, nA, loB,
                       nB);
  if (sel != 0)
    hipLaunchKernelGGL((sweep_adjoint<N, DIR, true>), g, b, 0, st, Uin, lam, dt, P, gfaces, floors, sel, loA, nA, loB,
                       nB);
  return hipGetLastError();
}

template <int N>
hipError_t sweep_adj_n(const DevPlan& P, const double* Uin, double* lam, const double* dt, const double* gfaces,
                       const unsigned long long* floors, int64_t floors_host, int dir, const int swept[3],
                       hipStream_t st) {
  if (dir == 0) return sweep_adj_nd<N, 0>(P, Uin, lam, dt, gfaces, floors, floors_host, swept, st);
  if (dir == 1) return sweep_adj_nd<N, 1>(P, Uin, lam, dt, gfaces, floors, floors_host, swept, st);
  return sweep_adj_nd<N, 2>(P, Uin, lam, dt, gfaces, floors, floors_host, swept, st);
}

template <int N, int NF>
hipError_t reflux_adj_nf(const DevPlan& P, const double* lam, const double* dt, double* gfaces, hipStream_t st) {
  for (int d = 0; d < 3; d++) {
    const int64_t n = P.nreflux[d] * N * N;
    if (n == 0) continue;
    const dim3 g(gridn(n, 256)), b(256);
    if (d == 0) hipLaunchKernelGGL((reflux_adjoint<N, 0, NF>), g, b, 0, st, lam, dt, P, gfaces);
    else if (d == 1) hipLaunchKernelGGL((reflux_adjoint<N, 1, NF>), g, b, 0, st, lam, dt, P, gfaces);
    else hipLaunchKernelGGL((reflux_adjoint<N, 2, NF>), g, b, 0, st, lam, dt, P, gfaces);
  }
  return hipGetLastError();
}

template <int N>
hipError_t reflux_adj_n(const DevPlan& P, const double* lam, const double* dt, double* gfaces, hipStream_t st) {
  return P.nf == kFieldsDE ? reflux_adj_nf<N, kFieldsDE>(P, lam, dt, gfaces, st)
                           : reflux_adj_nf<N, kFields>(P, lam, dt, gfaces, st);
}

template <int N, int NF>
hipError_t refresh_adj_nf(const DevPlan& P, double* lam, const double* Uref, hipStream_t st) {
  constexpr int M = N + 2 * G;
  constexpr int64_t GC = int64_t(M) * M * M - int64_t(N) * N * N;
  if (P.np2 > 0)
    hipLaunchKernelGGL((refresh2_adjoint<N, NF>), dim3(gridn(P.np2 * GC, 256)), dim3(256), 0, st, lam, Uref, P);
  if (P.nleaf > 0)
    hipLaunchKernelGGL((refresh1_adjoint<N, NF>), dim3(gridn(P.nleaf * GC, 256)), dim3(256), 0, st, lam, P);
  return hipGetLastError();
}

template <int N>
hipError_t refresh_adj_n(const DevPlan& P, double* lam, const double* Uref, hipStream_t st) {
  return P.nf == kFieldsDE ? refresh_adj_nf<N, kFieldsDE>(P, lam, Uref, st) : refresh_adj_nf<N, kFields>(P, lam, Uref, st);
}

}  // namespace

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero, dim3(gridn(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_reflux_adjoint(const DevPlan& P, const double* lam, const double* dt, double* gfaces,
                                 hipStream_t st) {
  switch (P.N) {
    case 8: return reflux_adj_n<8>(P, lam, dt, gfaces, st);
    case 16: return reflux_adj_n<16>(P, lam, dt, gfaces, st);
    case 32: return reflux_adj_n<32>(P, lam, dt, gfaces, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sweep_adjoint(const DevPlan& P, const double* Uin, double* lam, const double* dt,
                                const double* gfaces, const unsigned long long* floors, int64_t floors_host, int dir,
                                const int swept[3], hipStream_t st) {
  switch (P.N) {
    case 8: return sweep_adj_n<8>(P, Uin, lam, dt, gfaces, floors, floors_host, dir, swept, st);
    case 16: return sweep_adj_n<16>(P, Uin, lam, dt, gfaces, floors, floors_host, dir, swept, st);
    case 32: return sweep_adj_n<32>(P, Uin, lam, dt, gfaces, floors, floors_host, dir, swept, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_refresh_adjoint(const DevPlan& P, double* lam, const double* Uref, hipStream_t st) {
  switch (P.N) {
    case 8: return refresh_adj_n<8>(P, lam, Uref, st);
    case 16: return refresh_adj_n<16>(P, lam, Uref, st);
    case 32: return refresh_adj_n<32>(P, lam, Uref, st);
    default: return hipErrorInvalidValue;
  }
}

// Work items per leaf of the largest sweep-transpose launch: ceil(M^2 / R)
// tiles of WG lanes on each axis.
int64_t adjoint_items_per_leaf(int N) {
  auto items = [](auto shape) {
    using S = decltype(shape);
    return int64_t((S::M * S::M + S::R - 1) / S::R) * S::WG;
  };
  switch (N) {
    case 8: return std::max({items(AdjShape<8, 0>{}), items(AdjShape<8, 1>{}), items(AdjShape<8, 2>{})});
    case 16: return std::max({items(AdjShape<16, 0>{}), items(AdjShape<16, 1>{}), items(AdjShape<16, 2>{})});
    default: return std::max({items(AdjShape<32, 0>{}), items(AdjShape<32, 1>{}), items(AdjShape<32, 2>{})});
  }
}

}  // namespace amr
