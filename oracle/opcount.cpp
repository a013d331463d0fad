/*
 * opcount.cpp -- instrumented count of the FP64 operations the oracle executes.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE (part of the oracle).  It compiles the
 * oracle's own PPM pencil and cell update (ppm_pencil.inc, the code the
 * oracle's sweeps run) once more with `double` standing for a number type that
 * counts every addition, subtraction, multiplication, division and square
 * root it performs.  Negation, |x|, comparisons and selects are not counted,
 * as in the cost model of the benchmark.  Nothing here changes a value: each
 * counted operation is the same IEEE operation on the same operands.
 *
 * The count is of the operations as the oracle's formulas write them: a
 * subexpression the source evaluates twice counts twice, and a branch not
 * taken counts nothing, so the count depends on the data through the branch
 * choices (limiters, parabola cases, wave directions, shock or rarefaction).
 */
#include <cmath>
#include <cstdint>
#include <cstdlib>

#include "amr_oracle.h"

namespace {

struct OpCounts {
  int64_t add, sub, mul, div, sqrt;
};
thread_local OpCounts g_ops;

// An FP64 value whose arithmetic is counted.
struct Cd {
  double v;
  Cd() : v(0.0) {}
  Cd(double x) : v(x) {}  // NOLINT: literals and plain doubles enter implicitly
};
inline Cd operator+(Cd a, Cd b) { g_ops.add++; return Cd(a.v + b.v); }
inline Cd operator-(Cd a, Cd b) { g_ops.sub++; return Cd(a.v - b.v); }
inline Cd operator*(Cd a, Cd b) { g_ops.mul++; return Cd(a.v * b.v); }
inline Cd operator/(Cd a, Cd b) { g_ops.div++; return Cd(a.v / b.v); }
inline Cd operator-(Cd a) { return Cd(-a.v); }
inline bool operator<(Cd a, Cd b) { return a.v < b.v; }
inline bool operator>(Cd a, Cd b) { return a.v > b.v; }
inline bool operator<=(Cd a, Cd b) { return a.v <= b.v; }
inline bool operator>=(Cd a, Cd b) { return a.v >= b.v; }
inline bool operator!=(Cd a, Cd b) { return a.v != b.v; }
inline bool operator==(Cd a, Cd b) { return a.v == b.v; }
inline Cd sqrt(Cd a) { g_ops.sqrt++; return Cd(std::sqrt(a.v)); }
inline bool signbit(Cd a) { return std::signbit(a.v); }

// The includer's part of the oracle's interface (see ppm_pencil.inc): no
// planted mistakes and no branch tape, so every choice is the data's own.
const int g_debug = 0;
inline int BR(int c) { return c; }
inline Cd babs(Cd x) { return BR(signbit(x) != 0) ? -x : x; }
inline Cd dmax(Cd a, Cd b) { return BR(a < b) ? b : a; }
inline Cd dmin(Cd a, Cd b) { return BR(a < b) ? a : b; }

#define double Cd
#include "ppm_pencil.inc"
#undef double

void store(int64_t* out) {
  out[0] = g_ops.add;
  out[1] = g_ops.sub;
  out[2] = g_ops.mul;
  out[3] = g_ops.div;
  out[4] = g_ops.sqrt;
}

}  // namespace

extern "C" {

/* Operations of one sweep of a pencil of n cells, as the oracle's sweep runs
 * it: the fluxes at the n - 5 interfaces j + 1/2, j = 2 .. n - 4, then the
 * conservative update and floors of cells 3 .. n - 4.  U holds the five
 * conserved fields (rho, m_normal, m_t1, m_t2, E) field-major, n values each.
 * gas = (gamma, rho_floor, p_floor); iters is the fixed Newton count.  counts
 * receives (add, sub, mul, div, sqrt); returns the number of floor resets, or
 * -1 if n < 7. */
int orc_count_sweep_ops(const double* gas, int iters, double nu, int n, const double* U, int64_t* counts) {
  if (n < 7) return -1;
  const consts_t K = make_consts(gas[0], gas[1], gas[2], iters);
  Cd* u = static_cast<Cd*>(std::malloc(sizeof(Cd) * 5 * (size_t)n));
  Cd* f = static_cast<Cd*>(std::malloc(sizeof(Cd) * 5 * (size_t)(n - 5)));
  Cd* ug = static_cast<Cd*>(std::malloc(sizeof(Cd) * (size_t)(n - 5)));
  if (!u || !f || !ug) {
    std::free(u); std::free(f); std::free(ug);
    return -1;
  }
  for (int i = 0; i < 5 * n; i++) u[i] = Cd(U[i]);
  const Cd* in[5];
  Cd* out[5];
  for (int v = 0; v < 5; v++) {
    in[v] = u + (size_t)v * n;
    out[v] = f + (size_t)v * (n - 5);
  }
  g_ops = OpCounts{0, 0, 0, 0, 0};
  pencil(&K, Cd(nu), n, in, out, ug);
  int nfl = 0;
  for (int j = ORC_GHOST; j < n - ORC_GHOST; j++) {
    Cd Uc[6], Fm[6], Fp[6], Un[6];
    for (int v = 0; v < 5; v++) {
      Uc[v] = in[v][j];
      Fm[v] = out[v][j - ORC_GHOST];
      Fp[v] = out[v][j - ORC_GHOST + 1];
    }
    nfl += update_cell(&K, Cd(nu), Uc, Fm, Fp, ug[j - ORC_GHOST], ug[j - ORC_GHOST + 1], Un);
  }
  store(counts);
  std::free(u); std::free(f); std::free(ug);
  return nfl;
}

/* Operations of one Riemann solve (the two-shock solver of the pencil) on the
 * edge states WL, WR (rho, u, v, w, p); gas = (gamma, p_floor).  flux_out
 * receives the 5 fluxes, for the check that counting changes no value. */
void orc_count_riemann_ops(const double* gas, int iters, const double* WLs, const double* WRs, int64_t* counts,
                           double* flux_out) {
  const consts_t K = make_consts(gas[0], 0.0, gas[1], iters);
  Cd L[5], R[5], Wg[5], F[6];
  for (int v = 0; v < 5; v++) {
    L[v] = Cd(WLs[v]);
    R[v] = Cd(WRs[v]);
  }
  g_ops = OpCounts{0, 0, 0, 0, 0};
  riemann(&K, L, R, Wg, F, nullptr, nullptr);
  store(counts);
  for (int v = 0; v < 5; v++) flux_out[v] = F[v].v;
}

/* Operations of one building block of the sweep, for the pins of the cost
 * model.  which: 0 primitive recovery (in: rho, m_n, m_t1, m_t2, E); 1 limited
 * slope (in: q[j-1], q[j], q[j+1]); 2 parabola (in: q, qL, qR, f); 3
 * characteristic tracing of one cell (in: rho, m_n, m_t1, m_t2, E of the cell,
 * then (qL, qR, f) for each of the 5 primitives; nu); 4 cell update and floors
 * (in: the cell's 5 fields, the fluxes at its lower and upper faces).  gas =
 * (gamma, rho_floor, p_floor).  Only the block's own operations are counted:
 * its inputs (primitives, parabolas) are prepared before the count starts.
 * Returns 0, or -1 for an unknown block. */
int orc_count_block_ops(int which, const double* gas, double nu, const double* in, int64_t* counts) {
  const consts_t K = make_consts(gas[0], gas[1], gas[2], 1);
  switch (which) {
    case 0: {
      g_ops = OpCounts{0, 0, 0, 0, 0};
      (void)to_prim(&K, in[0], in[1], in[2], in[3], in[4], 0.0);
      break;
    }
    case 1: {
      g_ops = OpCounts{0, 0, 0, 0, 0};
      (void)mc_slope(in[0], in[1], in[2]);
      break;
    }
    case 2: {
      g_ops = OpCounts{0, 0, 0, 0, 0};
      (void)make_parabola(&K, in[0], in[1], in[2], in[3]);
      break;
    }
    case 3: {
      const prim_t C = to_prim(&K, in[0], in[1], in[2], in[3], in[4], 0.0);
      para_t par[5];
      for (int v = 0; v < 5; v++) par[v] = make_parabola(&K, C.q[v], in[5 + 3 * v], in[6 + 3 * v], in[7 + 3 * v]);
      Cd WL[5], WR[5];
      g_ops = OpCounts{0, 0, 0, 0, 0};
      trace_cell(&K, &C, par, Cd(nu), WL, WR);
      break;
    }
    case 4: {
      Cd Uc[6], Fm[6], Fp[6], Un[6];
      for (int v = 0; v < 5; v++) {
        Uc[v] = Cd(in[v]);
        Fm[v] = Cd(in[5 + v]);
        Fp[v] = Cd(in[10 + v]);
      }
      g_ops = OpCounts{0, 0, 0, 0, 0};
      (void)update_cell(&K, Cd(nu), Uc, Fm, Fp, Cd(0.0), Cd(0.0), Un);
      break;
    }
    default:
      return -1;
  }
  store(counts);
  return 0;
}

}  // extern "C"
