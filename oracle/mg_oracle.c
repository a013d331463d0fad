/*
 * mg_oracle.c -- plain FP64 CPU oracle of the mg0 Poisson solver.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke entry
 * point and the benchmark's CPU-baseline leg may load it.  It shares no code
 * with the HIP path.
 *
 * The paper (Sec. II-C) names mg0 as Enzo-P's geometric multigrid V-cycle
 * solver for the gravitational potential, used for self-gravity on a uniform
 * mesh of 32^3 blocks in its cosmology scaling test (Sec. III); it gives no
 * formulas.  Readings (a textbook cell-centred multigrid, Briggs, Henson and
 * McCormick, "A Multigrid Tutorial", 2nd ed., 2000; Trottenberg, Oosterlee and
 * Schueller, "Multigrid", 2001):
 *   - the problem: the 7-point Laplacian (sum of the 6 neighbours - 6 phi)
 *     / h^2 = f on a uniform periodic grid of nx x ny x nz cells of spacing
 *     h; f is first made mean-free, and the returned phi has zero mean;
 *   - levels: level l+1 halves every axis of level l, and exists while every
 *     axis of level l is a multiple of 4 (so every level has even sizes and a
 *     consistent red-black colouring across the periodic wrap); h doubles;
 *   - smoother: red-black Gauss-Seidel, red = (i + j + k) even first, each
 *     cell phi = (S - h^2 f) / 6 with S = ((W + E) + (S + N)) + (B + T) of
 *     the current neighbour values; nu1 sweeps before, nu2 after the coarse
 *     correction;
 *   - restriction: the coarse right-hand side is the mean of the residuals
 *     r = f - (S - 6 phi) / h^2 of the 8 children, summed x fastest, then
 *     y, then z, in pairs, times 1/8; the coarse correction starts from 0;
 *   - prolongation: trilinear between coarse cell centres: a fine cell adds
 *     (27 c + 9 ((cx + cy) + cz) + 3 ((cxy + cxz) + cyz) + cxyz) / 64 of the
 *     parent c and the coarse neighbours towards the fine cell's corner;
 *   - coarsest level: 64 red-black sweeps from 0;
 *   - a solve: f <- f - mean(f); residual L2 norm; then per V-cycle the
 *     cycle and the new norm; at the end phi <- phi - mean(phi).
 * Every sum is evaluated as parenthesised here; means are sequential sums
 * in index order divided by the count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "amr_oracle.h"

#define MG_MAXLEV 24
#define MG_COARSE_SWEEPS 64

/* Test-only switches that plant a known mistake (ORC_MG_DEBUG_*). */
static int g_mg_debug = 0;
void orc_mg_set_debug(int flags) { g_mg_debug = flags; }

typedef struct {
  int n[3];
  double h;
  double* phi;
  double* f;
} level_t;

static inline int64_t at(const level_t* L, int i, int j, int k) {
  i = (i + L->n[0]) % L->n[0];
  j = (j + L->n[1]) % L->n[1];
  k = (k + L->n[2]) % L->n[2];
  return ((int64_t)k * L->n[1] + j) * L->n[0] + i;
}

static inline double nbr_sum(const level_t* L, int i, int j, int k) {
  const double* p = L->phi;
  return ((p[at(L, i - 1, j, k)] + p[at(L, i + 1, j, k)]) + (p[at(L, i, j - 1, k)] + p[at(L, i, j + 1, k)])) +
         (p[at(L, i, j, k - 1)] + p[at(L, i, j, k + 1)]);
}

static double residual_at(const level_t* L, int i, int j, int k) {
  const int64_t c = at(L, i, j, k);
  const double ih2 = 1.0 / (L->h * L->h);
  return L->f[c] - (nbr_sum(L, i, j, k) - 6.0 * L->phi[c]) * ih2;
}

static void rbgs(level_t* L) {
  const double h2 = L->h * L->h, sixth = 1.0 / 6.0;
  for (int color = 0; color < 2; color++)
    for (int k = 0; k < L->n[2]; k++)
      for (int j = 0; j < L->n[1]; j++)
        for (int i = 0; i < L->n[0]; i++) {
          if (((i + j + k) & 1) != color) continue;
          const int64_t c = at(L, i, j, k);
          L->phi[c] = (g_mg_debug & ORC_MG_DEBUG_SMOOTH_SIGN) ? (nbr_sum(L, i, j, k) + h2 * L->f[c]) * sixth
                                                               : (nbr_sum(L, i, j, k) - h2 * L->f[c]) * sixth;
        }
}

static void restrict_residual(const level_t* F, level_t* C) {
  for (int k = 0; k < C->n[2]; k++)
    for (int j = 0; j < C->n[1]; j++)
      for (int i = 0; i < C->n[0]; i++) {
        double r[8];
        for (int o = 0; o < 8; o++) r[o] = residual_at(F, 2 * i + (o & 1), 2 * j + ((o >> 1) & 1), 2 * k + (o >> 2));
        const int64_t c = at(C, i, j, k);
        C->f[c] = (((r[0] + r[1]) + (r[2] + r[3])) + ((r[4] + r[5]) + (r[6] + r[7]))) *
                  ((g_mg_debug & ORC_MG_DEBUG_RESTRICT_SUM) ? 1.0 : 0.125);
        C->phi[c] = 0.0;
      }
}

static void prolong_add(const level_t* C, level_t* F) {
  const double w64 = 1.0 / 64.0;
  for (int k = 0; k < F->n[2]; k++)
    for (int j = 0; j < F->n[1]; j++)
      for (int i = 0; i < F->n[0]; i++) {
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
        const double* p = C->phi;
        const double c0 = p[at(C, I, J, K)];
        const double cx = p[at(C, I + si, J, K)], cy = p[at(C, I, J + sj, K)], cz = p[at(C, I, J, K + sk)];
        const double cxy = p[at(C, I + si, J + sj, K)], cxz = p[at(C, I + si, J, K + sk)],
                     cyz = p[at(C, I, J + sj, K + sk)];
        const double cxyz = p[at(C, I + si, J + sj, K + sk)];
        double v = ((27.0 * c0 + 9.0 * ((cx + cy) + cz)) + (3.0 * ((cxy + cxz) + cyz) + cxyz)) * w64;
        if (g_mg_debug & ORC_MG_DEBUG_INJECT) v = c0;
        F->phi[at(F, i, j, k)] += v;
      }
}

static void vcycle(level_t* Ls, int l, int nl, int nu1, int nu2) {
  if (l == nl - 1) {
    for (int s = 0; s < MG_COARSE_SWEEPS; s++) rbgs(&Ls[l]);
    return;
  }
  for (int s = 0; s < nu1; s++) rbgs(&Ls[l]);
  restrict_residual(&Ls[l], &Ls[l + 1]);
  vcycle(Ls, l + 1, nl, nu1, nu2);
  prolong_add(&Ls[l + 1], &Ls[l]);
  for (int s = 0; s < nu2; s++) rbgs(&Ls[l]);
}

static double mean(const double* a, int64_t n) {
  double s = 0.0;
  for (int64_t q = 0; q < n; q++) s += a[q];
  return s / (double)n;
}

static double resid_norm(const level_t* L) {
  double s = 0.0;
  for (int k = 0; k < L->n[2]; k++)
    for (int j = 0; j < L->n[1]; j++)
      for (int i = 0; i < L->n[0]; i++) {
        const double r = residual_at(L, i, j, k);
        s += r * r;
      }
  return sqrt(s);
}

int orc_mg_levels(int nx, int ny, int nz) {
  int n[3] = {nx, ny, nz}, nl = 1;
  while (nl < MG_MAXLEV && n[0] % 4 == 0 && n[1] % 4 == 0 && n[2] % 4 == 0) {
    for (int a = 0; a < 3; a++) n[a] /= 2;
    nl++;
  }
  return nl;
}

int orc_mg_solve(int nx, int ny, int nz, double h, const double* f, double* phi, int ncycles, int nu1, int nu2,
                 double* resid) {
  if (nx < 2 || ny < 2 || nz < 2 || nx % 2 || ny % 2 || nz % 2 || !(h > 0.0) || ncycles < 0 || nu1 < 0 || nu2 < 0)
    return -1;
  const int nl = orc_mg_levels(nx, ny, nz);
  level_t Ls[MG_MAXLEV];
  int n[3] = {nx, ny, nz};
  double hl = h;
  for (int l = 0; l < nl; l++) {
    const int64_t cnt = (int64_t)n[0] * n[1] * n[2];
    memcpy(Ls[l].n, n, sizeof n);
    Ls[l].h = hl;
    Ls[l].phi = (double*)calloc((size_t)cnt, sizeof(double));
    Ls[l].f = (double*)calloc((size_t)cnt, sizeof(double));
    for (int a = 0; a < 3; a++) n[a] /= 2;
    hl = 2.0 * hl;
  }
  const int64_t n0 = (int64_t)nx * ny * nz;
  const double fm = mean(f, n0);
  for (int64_t q = 0; q < n0; q++) {
    Ls[0].f[q] = f[q] - fm;
    Ls[0].phi[q] = phi[q];
  }
  if (resid) resid[0] = resid_norm(&Ls[0]);
  for (int c = 0; c < ncycles; c++) {
    vcycle(Ls, 0, nl, nu1, nu2);
    if (resid) resid[c + 1] = resid_norm(&Ls[0]);
  }
  const double pm = mean(Ls[0].phi, n0);
  for (int64_t q = 0; q < n0; q++) phi[q] = Ls[0].phi[q] - pm;
  for (int l = 0; l < nl; l++) {
    free(Ls[l].phi);
    free(Ls[l].f);
  }
  return nl;
}

/* One V(nu1, nu2) cycle from phi = 0 on f as given (no mean handling): the
 * coarse-grid correction the composite solver takes on its root level. */
int orc_mg_vcycle_from_zero(int nx, int ny, int nz, double h, const double* f, double* phi, int nu1, int nu2) {
  if (nx < 2 || ny < 2 || nz < 2 || nx % 2 || ny % 2 || nz % 2 || !(h > 0.0)) return -1;
  const int nl = orc_mg_levels(nx, ny, nz);
  level_t Ls[MG_MAXLEV];
  int n[3] = {nx, ny, nz};
  double hl = h;
  for (int l = 0; l < nl; l++) {
    const int64_t cnt = (int64_t)n[0] * n[1] * n[2];
    memcpy(Ls[l].n, n, sizeof n);
    Ls[l].h = hl;
    Ls[l].phi = (double*)calloc((size_t)cnt, sizeof(double));
    Ls[l].f = (double*)calloc((size_t)cnt, sizeof(double));
    for (int a = 0; a < 3; a++) n[a] /= 2;
    hl = 2.0 * hl;
  }
  const int64_t n0 = (int64_t)nx * ny * nz;
  memcpy(Ls[0].f, f, (size_t)n0 * sizeof(double));
  vcycle(Ls, 0, nl, nu1, nu2);
  memcpy(phi, Ls[0].phi, (size_t)n0 * sizeof(double));
  for (int l = 0; l < nl; l++) {
    free(Ls[l].phi);
    free(Ls[l].f);
  }
  return nl;
}

/* Test hooks on the building blocks. */
void orc_mg_prolong_add(int nxc, int nyc, int nzc, const double* coarse, double* fine) {
  level_t C = {{nxc, nyc, nzc}, 1.0, (double*)coarse, NULL};
  level_t F = {{2 * nxc, 2 * nyc, 2 * nzc}, 0.5, fine, NULL};
  prolong_add(&C, &F);
}

void orc_mg_restrict_residual(int nx, int ny, int nz, double h, const double* f, const double* phi, double* coarse_f) {
  const int64_t nc = (int64_t)(nx / 2) * (ny / 2) * (nz / 2);
  double* cphi = (double*)calloc((size_t)nc, sizeof(double));
  level_t F = {{nx, ny, nz}, h, (double*)phi, (double*)f};
  level_t C = {{nx / 2, ny / 2, nz / 2}, 2.0 * h, cphi, coarse_f};
  restrict_residual(&F, &C);
  free(cphi);
}
