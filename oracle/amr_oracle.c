/*
 * amr_oracle.c -- plain FP64 CPU oracle of one AMR hydro timestep.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke entry
 * point and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header, table or constant generator with the HIP path; both follow the same
 * written readings of the paper.
 *
 * What the paper fixes (Bordner & Norman, Sec. II-B and II-C):
 *   - the mesh is an array of octrees; each octree node is a Block of N^3
 *     cells; leaves carry the solution;
 *   - before a Method runs on a Block its ghost layer of the stated width is
 *     refreshed from neighbouring Blocks, with Restrict (fine -> coarse) and
 *     Prolong (coarse -> fine) across refinement jumps;
 *   - the hydro Method is a modified piecewise-parabolic method (PPM).
 * Everything else is a reading, stated at the code that applies it:
 *   R-order : every formula is evaluated exactly as parenthesised; only
 *             + - * / sqrt and comparisons; max/min written as selects;
 *             built with -ffp-contract=off (no fused multiply-add).
 *   R-mesh  : cubic cells, dx_l = 1 / (Rx * N * 2^l); 2:1 balance across all
 *             26 neighbour directions; ghost width 3.
 *   R-order-of-refresh : phase 1 = same-level copies, restriction into
 *             coarse ghosts, outflow clamps; phase 2 = prolongation into
 *             fine ghosts (reads the coarse block's active + phase-1 cells).
 *   R-split : one refresh per step; sweeps x,y,z on even steps, z,y,x on
 *             odd; sweep s updates cells active along the axes swept so far
 *             (including this one) and all cells along the others.
 *   R-dt    : one dt per mesh per step from the CFL condition at step start.
 *   R-reflux: coarse cells next to a coarse-fine face take the area mean of
 *             the fine face fluxes, applied after the third sweep.
 * The oracle is single-threaded in semantics; OpenMP only splits loops over
 * blocks whose iterations are independent, so results do not depend on the
 * thread count.
 */
#include "amr_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define G ORC_GHOST

enum { ABSENT = 0, LEAF = 1, REFINED = 2 };

struct orc_mesh {
  orc_desc d;
  int N, M, nlev;
  int ext[ORC_MAXLEV][3];
  unsigned char* state[ORC_MAXLEV];
  int32_t* leaf_at[ORC_MAXLEV];
  int64_t nleaf;
  int32_t* key;   /* (level, i, j, k) per leaf */
  int nf;         /* fields per cell: 5, or 6 with the dual-energy field */
  double* U;      /* nleaf * nf * M^3 */
  double** face;  /* 6 per leaf: coarse-fine face flux buffers or NULL */
  int64_t floors;
};

static char g_err[256];
/* Test-only switches that plant a known mistake, to show that a pin fails
 * without the piece it checks (ORC_DEBUG_*). */
static int g_debug = 0;
const char* orc_last_error(void) { return g_err; }
static int fail(const char* msg) {
  snprintf(g_err, sizeof g_err, "%s", msg);
  return -1;
}

/* ------------------------------------------------------------------ */
/* Frozen-branch forward (the adjoint's reading: every discrete choice    */
/* held at the forward run's)                                             */
/* ------------------------------------------------------------------ */
/* A step's discrete choices -- limiter selections, the signs of |x|, the
 * parabola cases, the flattening switch and clamps, the wave-speed gates of
 * the tracing, the Riemann solver's floors, side, wave type and sampling
 * region, the prolongation's minmod, the positivity floors -- pass through
 * BR().  With no tape BR() returns its argument.  A recording tape stores
 * each choice in order; a replaying tape returns the stored choices instead,
 * so a perturbed run evaluates the same smooth branch of the scheme as the
 * recorded one and its central differences converge to the derivative the
 * adjoint takes.  While a tape is attached the step's loops run serially,
 * so the choices occur in one fixed order. */
typedef struct {
  unsigned char* b;
  int64_t n, cap, pos;
  int replay, overrun;
} tape_t;
static _Thread_local tape_t* t_tape = NULL;

static int BR(int c) {
  tape_t* t = t_tape;
  if (!t) return c;
  if (t->replay) {
    if (t->pos < t->n) return t->b[t->pos++];
    t->overrun = 1;
    return c;
  }
  if (t->n == t->cap) {
    int64_t cap = t->cap ? 2 * t->cap : (int64_t)1 << 20;
    unsigned char* nb = (unsigned char*)realloc(t->b, (size_t)cap);
    if (!nb) { t->overrun = 1; return c; }
    t->b = nb;
    t->cap = cap;
  }
  t->b[t->n++] = (unsigned char)(c != 0);
  return c;
}
/* |x| with its sign choice recorded (the same value as fabs) */
static inline double babs(double x) { return BR(signbit(x) != 0) ? -x : x; }
#define SERIAL_IF_TAPED if (t_tape == NULL)

static inline double dmax(double a, double b) { return BR(a < b) ? b : a; }
static inline double dmin(double a, double b) { return BR(a < b) ? a : b; }

/* The PPM pencil, the cell update and the gas constants they use; compiled
 * a second time with a counting number type by opcount.cpp. */
#include "ppm_pencil.inc"

static consts_t mesh_consts(const orc_mesh* m) {
  consts_t K = make_consts(m->d.gamma, m->d.rho_floor, m->d.p_floor, m->d.riemann_iters);
  K.de = m->d.dual_energy != 0;
  K.eta1 = m->d.eta1;
  K.eta2 = m->d.eta2;
  return K;
}

/* ------------------------------------------------------------------ */
/* Mesh: dense per-level node state, 2:1 balance                       */
/* ------------------------------------------------------------------ */

static inline int64_t nidx(const orc_mesh* m, int l, int i, int j, int k) {
  return ((int64_t)k * m->ext[l][1] + j) * m->ext[l][0] + i;
}
static inline int64_t cell(int M, int f, int a, int b, int c) {
  return (((int64_t)f * M + c) * M + b) * M + a;
}
static inline double* block_ptr(const orc_mesh* m, int64_t leaf) {
  return m->U + leaf * (int64_t)m->nf * m->M * m->M * m->M;
}
/* dx at level l: cubic cells, the x extent of the domain is 1. */
static inline double dx_level(const orc_mesh* m, int l) {
  return 1.0 / (double)((int64_t)m->d.root[0] * m->N << l);
}

static void refine_node(orc_mesh* m, int l, int i, int j, int k) {
  m->state[l][nidx(m, l, i, j, k)] = REFINED;
  for (int c = 0; c < 8; c++)
    m->state[l + 1][nidx(m, l + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + (c >> 2))] = LEAF;
}

/* Map a level-l block coordinate into the domain along axis ax: periodic
 * axes wrap, outflow axes have no block outside.  Returns 0 if outside. */
static int wrap_block(const orc_mesh* m, int l, int ax, int* v) {
  int e = m->ext[l][ax];
  if (*v >= 0 && *v < e) return 1;
  if (m->d.bc[ax] != ORC_BC_PERIODIC) return 0;
  *v = ((*v % e) + e) % e;
  return 1;
}

/* Level of the leaf covering level-l block position p (or l if the node at
 * level l exists, leaf or refined).  p is replaced by that node's position. */
static int covering_level(const orc_mesh* m, int l, int p[3]) {
  while (m->state[l][nidx(m, l, p[0], p[1], p[2])] == ABSENT) {
    l--;
    p[0] >>= 1; p[1] >>= 1; p[2] >>= 1;
  }
  return l;
}

/* 2:1 balance across faces, edges and corners: refine any leaf that is two
 * or more levels coarser than a leaf it touches, until none is. */
static void balance(orc_mesh* m) {
  int changed = 1;
  while (changed) {
    changed = 0;
    for (int l = 2; l < m->nlev; l++)
      for (int k = 0; k < m->ext[l][2]; k++)
        for (int j = 0; j < m->ext[l][1]; j++)
          for (int i = 0; i < m->ext[l][0]; i++) {
            if (m->state[l][nidx(m, l, i, j, k)] != LEAF) continue;
            for (int dz = -1; dz <= 1; dz++)
              for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                  if (!dx && !dy && !dz) continue;
                  int p[3] = {i + dx, j + dy, k + dz};
                  if (!wrap_block(m, l, 0, &p[0]) || !wrap_block(m, l, 1, &p[1]) ||
                      !wrap_block(m, l, 2, &p[2]))
                    continue;
                  int lv = covering_level(m, l, p);
                  if (l - lv >= 2) {
                    refine_node(m, lv, p[0], p[1], p[2]);
                    changed = 1;
                  }
                }
          }
  }
}

static int check_desc(const orc_desc* d) {
  if (d->block_cells < 8 || d->block_cells % 2) return fail("block_cells must be even and >= 8");
  if (d->max_level < 0 || d->max_level >= ORC_MAXLEV) return fail("max_level out of range");
  for (int a = 0; a < 3; a++) {
    if (d->root[a] < 1) return fail("root extent must be >= 1");
    if (d->bc[a] != ORC_BC_PERIODIC && d->bc[a] != ORC_BC_OUTFLOW) return fail("bad bc");
  }
  if (!(d->gamma > 1.0)) return fail("gamma must exceed 1");
  if (d->riemann_iters < 0) return fail("riemann_iters < 0");
  if (d->dual_energy != 0 && d->dual_energy != 1) return fail("dual_energy must be 0 or 1");
  if (d->dual_energy && !(d->eta1 >= 0.0 && d->eta1 <= 1.0 && d->eta2 >= 0.0 && d->eta2 <= 1.0))
    return fail("eta1 and eta2 must lie in [0, 1]");
  return 0;
}

static orc_mesh* alloc_mesh(const orc_desc* d) {
  orc_mesh* m = (orc_mesh*)calloc(1, sizeof(orc_mesh));
  m->d = *d;
  m->d.refine = NULL;
  m->d.n_refine = 0;
  m->N = d->block_cells;
  m->M = m->N + 2 * G;
  m->nf = d->dual_energy ? ORC_NFIELD + 1 : ORC_NFIELD;
  m->nlev = d->max_level + 1;
  for (int l = 0; l < m->nlev; l++) {
    for (int a = 0; a < 3; a++) m->ext[l][a] = d->root[a] << l;
    int64_t n = (int64_t)m->ext[l][0] * m->ext[l][1] * m->ext[l][2];
    m->state[l] = (unsigned char*)calloc((size_t)n, 1);
    m->leaf_at[l] = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  }
  return m;
}

void orc_destroy(orc_mesh* m) {
  if (!m) return;
  for (int l = 0; l < m->nlev; l++) {
    free(m->state[l]);
    free(m->leaf_at[l]);
  }
  if (m->face) {
    for (int64_t s = 0; s < 6 * m->nleaf; s++) free(m->face[s]);
    free(m->face);
  }
  free(m->key);
  free(m->U);
  free(m);
}

/* Number leaves (level, then z, y, x), allocate state and face buffers. */
static int finish_mesh(orc_mesh* m) {
  int64_t n = 0;
  for (int l = 0; l < m->nlev; l++) {
    int64_t cnt = (int64_t)m->ext[l][0] * m->ext[l][1] * m->ext[l][2];
    for (int64_t q = 0; q < cnt; q++) {
      m->leaf_at[l][q] = -1;
      if (m->state[l][q] == LEAF) n++;
    }
  }
  m->nleaf = n;
  m->key = (int32_t*)malloc((size_t)(4 * n) * sizeof(int32_t));
  n = 0;
  int uniform = 1;
  for (int l = 0; l < m->nlev; l++)
    for (int k = 0; k < m->ext[l][2]; k++)
      for (int j = 0; j < m->ext[l][1]; j++)
        for (int i = 0; i < m->ext[l][0]; i++)
          if (m->state[l][nidx(m, l, i, j, k)] == LEAF) {
            m->leaf_at[l][nidx(m, l, i, j, k)] = (int32_t)n;
            m->key[4 * n] = l; m->key[4 * n + 1] = i; m->key[4 * n + 2] = j; m->key[4 * n + 3] = k;
            if (l) uniform = 0;
            n++;
          }
  for (int a = 0; a < 3; a++)
    if (m->d.bc[a] == ORC_BC_OUTFLOW && !uniform)
      return fail("outflow boundaries are supported on single-level meshes only");
  int64_t M3 = (int64_t)m->M * m->M * m->M;
  m->U = (double*)calloc((size_t)(m->nleaf * m->nf * M3), sizeof(double));
  if (!m->U) return fail("out of memory");
  /* Coarse-fine faces: a face whose same-level neighbour position is refined
   * (this leaf is the coarse side) or absent (this leaf is the fine side). */
  m->face = (double**)calloc((size_t)(6 * m->nleaf), sizeof(double*));
  for (int64_t s = 0; s < m->nleaf; s++) {
    const int32_t* kk = m->key + 4 * s;
    int l = kk[0];
    for (int dir = 0; dir < 3; dir++)
      for (int side = 0; side < 2; side++) {
        int p[3] = {kk[1], kk[2], kk[3]};
        p[dir] += side ? 1 : -1;
        if (!wrap_block(m, l, dir, &p[dir])) continue;
        unsigned char st = m->state[l][nidx(m, l, p[0], p[1], p[2])];
        if (st != LEAF)
          m->face[6 * s + 2 * dir + side] =
              (double*)calloc((size_t)m->nf * m->N * m->N, sizeof(double));
      }
  }
  return 0;
}

int orc_create(const orc_desc* d, orc_mesh** out) {
  *out = NULL;
  if (check_desc(d)) return -1;
  orc_mesh* m = alloc_mesh(d);
  for (int64_t q = 0; q < (int64_t)m->ext[0][0] * m->ext[0][1] * m->ext[0][2]; q++) m->state[0][q] = LEAF;
  /* Static refinement list, applied in order; refining a node also refines
   * any leaf ancestor first. */
  for (int r = 0; r < d->n_refine; r++) {
    const int32_t* e = d->refine + 4 * r;
    int l = e[0];
    if (l < 0 || l >= d->max_level) { orc_destroy(m); return fail("refine level out of range"); }
    for (int a = 0; a < 3; a++)
      if (e[1 + a] < 0 || e[1 + a] >= m->ext[l][a]) { orc_destroy(m); return fail("refine key out of range"); }
    for (int a = 0; a <= l; a++) {
      int s = l - a;
      int i = e[1] >> s, j = e[2] >> s, k = e[3] >> s;
      if (m->state[a][nidx(m, a, i, j, k)] == LEAF) refine_node(m, a, i, j, k);
    }
  }
  balance(m);
  if (finish_mesh(m)) { orc_destroy(m); return -1; }
  *out = m;
  return 0;
}

int orc_create_from_leaves(const orc_desc* d, int64_t n, const int32_t* keys, orc_mesh** out) {
  *out = NULL;
  if (check_desc(d)) return -1;
  orc_mesh* m = alloc_mesh(d);
  for (int64_t s = 0; s < n; s++) {
    const int32_t* e = keys + 4 * s;
    int l = e[0];
    if (l < 0 || l > d->max_level) { orc_destroy(m); return fail("leaf level out of range"); }
    for (int a = 0; a < 3; a++)
      if (e[1 + a] < 0 || e[1 + a] >= m->ext[l][a]) { orc_destroy(m); return fail("leaf key out of range"); }
    unsigned char* st = &m->state[l][nidx(m, l, e[1], e[2], e[3])];
    if (*st != ABSENT) { orc_destroy(m); return fail("duplicate or overlapping leaf"); }
    *st = LEAF;
    for (int a = l - 1; a >= 0; a--) {
      int s2 = l - a;
      unsigned char* pa = &m->state[a][nidx(m, a, e[1] >> s2, e[2] >> s2, e[3] >> s2)];
      if (*pa == LEAF) { orc_destroy(m); return fail("leaf inside another leaf"); }
      *pa = REFINED;
    }
  }
  /* Every root covered and every refined node has all eight children. */
  for (int l = 0; l < m->nlev; l++)
    for (int k = 0; k < m->ext[l][2]; k++)
      for (int j = 0; j < m->ext[l][1]; j++)
        for (int i = 0; i < m->ext[l][0]; i++) {
          unsigned char st = m->state[l][nidx(m, l, i, j, k)];
          if (l == 0 && st == ABSENT) { orc_destroy(m); return fail("root not covered"); }
          if (st == REFINED) {
            if (l + 1 >= m->nlev) { orc_destroy(m); return fail("refined node at max level"); }
            for (int c = 0; c < 8; c++)
              if (m->state[l + 1][nidx(m, l + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + (c >> 2))] == ABSENT) {
                orc_destroy(m);
                return fail("leaves do not tile the domain");
              }
          }
        }
  /* 2:1 balance must already hold. */
  for (int l = 2; l < m->nlev; l++)
    for (int k = 0; k < m->ext[l][2]; k++)
      for (int j = 0; j < m->ext[l][1]; j++)
        for (int i = 0; i < m->ext[l][0]; i++) {
          if (m->state[l][nidx(m, l, i, j, k)] != LEAF) continue;
          for (int q = 0; q < 27; q++) {
            if (q == 13) continue;
            int p[3] = {i + q % 3 - 1, j + (q / 3) % 3 - 1, k + q / 9 - 1};
            if (!wrap_block(m, l, 0, &p[0]) || !wrap_block(m, l, 1, &p[1]) || !wrap_block(m, l, 2, &p[2]))
              continue;
            if (l - covering_level(m, l, p) >= 2) { orc_destroy(m); return fail("leaves violate 2:1 balance"); }
          }
        }
  if (finish_mesh(m)) { orc_destroy(m); return -1; }
  *out = m;
  return 0;
}

int64_t orc_nleaf(const orc_mesh* m) { return m->nleaf; }
int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_leaf_keys(const orc_mesh* m, int32_t* out) {
  memcpy(out, m->key, (size_t)(4 * m->nleaf) * sizeof(int32_t));
}
double* orc_state(orc_mesh* m) { return m->U; }
int64_t orc_floor_count(const orc_mesh* m) { return m->floors; }
int orc_nfields(const orc_mesh* m) { return m->nf; }

/* ------------------------------------------------------------------ */
/* Ghost refresh (Sec. II-B: ghost layer of width 3 for all 5 fields)  */
/* ------------------------------------------------------------------ */

/* Boundary condition on a level-l global cell index along axis ax:
 * periodic wraps, outflow clamps to the nearest domain cell. */
static int64_t bc_cell(const orc_mesh* m, int l, int ax, int64_t p) {
  int64_t n = (int64_t)m->ext[l][ax] * m->N;
  if (p >= 0 && p < n) return p;
  if (m->d.bc[ax] == ORC_BC_PERIODIC) return ((p % n) + n) % n;
  return p < 0 ? 0 : n - 1;
}

static inline int is_active(int N, int a, int b, int c) {
  return a >= G && a < G + N && b >= G && b < G + N && c >= G && c < G + N;
}

/* Value of the cell at level-l global index q inside the leaf that holds it
 * (q's block must be a leaf at level l). */
static inline double leaf_value_of(const orc_mesh* m, const double* data, int nf, int l, const int64_t q[3],
                                   int f) {
  int N = m->N;
  int bx = (int)(q[0] / N), by = (int)(q[1] / N), bz = (int)(q[2] / N);
  int32_t s = m->leaf_at[l][nidx(m, l, bx, by, bz)];
  const double* B = data + s * (int64_t)nf * m->M * m->M * m->M;
  return B[cell(m->M, f, (int)(q[0] - (int64_t)bx * N) + G, (int)(q[1] - (int64_t)by * N) + G,
                (int)(q[2] - (int64_t)bz * N) + G)];
}
static inline double leaf_value(const orc_mesh* m, int l, const int64_t q[3], int f) {
  return leaf_value_of(m, m->U, m->nf, l, q, f);
}

/* Restrict (Sec. II-B): the coarse value is the mean of its 8 children,
 * summed pairwise in the fixed order x fastest, then y, then z. */
static double restrict8(const double v[8]) {
  return (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) * 0.125;
}

/* minmod(a,b): the smaller-magnitude argument if both have the same sign,
 * else 0 (ties take b). */
static inline double minmod(double a, double b) {
  return BR(a * b > 0.0) ? (BR(babs(a) < babs(b)) ? a : b) : 0.0;
}

/* Ghost refresh of nf fields stored like the state (per leaf nf x M^3).
 * linear = 0: the minmod-limited prolongation above (hydro); linear = 1:
 * unlimited central slopes s_d = 0.5 (U_{P+e_d} - U_{P-e_d}), the linear
 * interpolation of the composite Poisson operator. */
static void refresh_fields(const orc_mesh* m, double* data, int nf, int phase, int linear) {
  const int N = m->N, M = m->M;
#pragma omp parallel for schedule(dynamic, 1) SERIAL_IF_TAPED
  for (int64_t s = 0; s < m->nleaf; s++) {
    const int32_t* kk = m->key + 4 * s;
    const int l = kk[0];
    double* B = data + s * (int64_t)nf * M * M * M;
    for (int c = 0; c < M; c++)
      for (int b = 0; b < M; b++)
        for (int a = 0; a < M; a++) {
          if (is_active(N, a, b, c)) continue;
          int64_t p[3] = {(int64_t)kk[1] * N + a - G, (int64_t)kk[2] * N + b - G, (int64_t)kk[3] * N + c - G};
          for (int ax = 0; ax < 3; ax++) p[ax] = bc_cell(m, l, ax, p[ax]);
          int bp[3] = {(int)(p[0] / N), (int)(p[1] / N), (int)(p[2] / N)};
          unsigned char st = m->state[l][nidx(m, l, bp[0], bp[1], bp[2])];
          if (phase == 1 && st == LEAF) {
            for (int f = 0; f < nf; f++) B[cell(M, f, a, b, c)] = leaf_value_of(m, data, nf, l, p, f);
          } else if (phase == 1 && st == REFINED) {
            for (int f = 0; f < nf; f++) {
              double v[8];
              for (int o = 0; o < 8; o++) {
                int64_t q[3] = {2 * p[0] + (o & 1), 2 * p[1] + ((o >> 1) & 1), 2 * p[2] + (o >> 2)};
                v[o] = leaf_value_of(m, data, nf, l + 1, q, f);
              }
              B[cell(M, f, a, b, c)] = restrict8(v);
            }
          } else if (phase == 2 && st == ABSENT) {
            /* Prolong (Sec. II-B): parent value plus limited slopes times the
             * octant offsets, U_f = ((U_P + 0.25 o_x s_x) + 0.25 o_y s_y)
             * + 0.25 o_z s_z, s_d = minmod(U_{P+e_d} - U_P, U_P - U_{P-e_d}),
             * read from the coarse leaf's active and phase-1 ghost cells. */
            int64_t pc[3] = {p[0] >> 1, p[1] >> 1, p[2] >> 1};
            int cb[3] = {(int)(pc[0] / N), (int)(pc[1] / N), (int)(pc[2] / N)};
            int32_t sc = m->leaf_at[l - 1][nidx(m, l - 1, cb[0], cb[1], cb[2])];
            const double* C = data + sc * (int64_t)nf * M * M * M;
            int lc[3];
            double o[3];
            for (int ax = 0; ax < 3; ax++) {
              lc[ax] = (int)(pc[ax] - (int64_t)cb[ax] * N) + G;
              o[ax] = (p[ax] & 1) ? 1.0 : -1.0;
            }
            for (int f = 0; f < nf; f++) {
              double u0 = C[cell(M, f, lc[0], lc[1], lc[2])];
              double sl[3];
              if (linear == 2) {
                sl[0] = sl[1] = sl[2] = 0.0;
              } else if (linear) {
                sl[0] = 0.5 * (C[cell(M, f, lc[0] + 1, lc[1], lc[2])] - C[cell(M, f, lc[0] - 1, lc[1], lc[2])]);
                sl[1] = 0.5 * (C[cell(M, f, lc[0], lc[1] + 1, lc[2])] - C[cell(M, f, lc[0], lc[1] - 1, lc[2])]);
                sl[2] = 0.5 * (C[cell(M, f, lc[0], lc[1], lc[2] + 1)] - C[cell(M, f, lc[0], lc[1], lc[2] - 1)]);
              } else {
                sl[0] = minmod(C[cell(M, f, lc[0] + 1, lc[1], lc[2])] - u0, u0 - C[cell(M, f, lc[0] - 1, lc[1], lc[2])]);
                sl[1] = minmod(C[cell(M, f, lc[0], lc[1] + 1, lc[2])] - u0, u0 - C[cell(M, f, lc[0], lc[1] - 1, lc[2])]);
                sl[2] = minmod(C[cell(M, f, lc[0], lc[1], lc[2] + 1)] - u0, u0 - C[cell(M, f, lc[0], lc[1], lc[2] - 1)]);
              }
              B[cell(M, f, a, b, c)] =
                  ((u0 + (0.25 * o[0]) * sl[0]) + (0.25 * o[1]) * sl[1]) + (0.25 * o[2]) * sl[2];
            }
          }
        }
  }
}

static void refresh_phase(orc_mesh* m, int phase) { refresh_fields(m, m->U, m->nf, phase, 0); }

void orc_refresh(orc_mesh* m) {
  refresh_phase(m, 1);
  refresh_phase(m, 2);
}

/* ------------------------------------------------------------------ */
/* CFL time step                                                        */
/* ------------------------------------------------------------------ */

/* dt = C_cfl * min over active leaf cells of dx_l / (max_d |u_d| + c); the
 * min over d of dx/(|u_d|+c) equals this because correctly rounded + and /
 * are monotone.  Primitive recovery as in the sweeps, x,y,z order. */
static double cfl_min(const orc_mesh* m) {
  const consts_t K = mesh_consts(m);
  const int N = m->N, M = m->M;
  double best = INFINITY;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : best)
  for (int64_t s = 0; s < m->nleaf; s++) {
    const double* B = block_ptr(m, s);
    const double dx = dx_level(m, m->key[4 * s]);
    for (int c = G; c < G + N; c++)
      for (int b = G; b < G + N; b++)
        for (int a = G; a < G + N; a++) {
          double rho = B[cell(M, 0, a, b, c)];
          double ir = 1.0 / rho;
          double u = B[cell(M, 1, a, b, c)] * ir, v = B[cell(M, 2, a, b, c)] * ir,
                 w = B[cell(M, 3, a, b, c)] * ir;
          double p = cell_pressure(&K, rho, u, v, w, B[cell(M, 4, a, b, c)],
                                   K.de ? B[cell(M, 5, a, b, c)] : 0.0);
          p = p < K.p_floor ? K.p_floor : p;
          double cs = sqrt((K.gamma * p) * ir);
          double vm = (g_debug & ORC_DEBUG_CFL_SUM) ? (fabs(u) + fabs(v)) + fabs(w)
                                                    : dmax(dmax(fabs(u), fabs(v)), fabs(w));
          double t = dx / (vm + cs);
          best = t < best ? t : best;
        }
  }
  return best;
}

double orc_cfl_dt(const orc_mesh* m) { return m->d.cfl * cfl_min(m); }

/* One directional sweep over every leaf.  swept[a] says whether axis a was
 * already swept this step (then only its active range is updated). */
static void sweep(orc_mesh* m, const consts_t* K, int dir, const int swept[3], double dt) {
  const int N = m->N, M = m->M;
  const int t1 = (dir + 1) % 3, t2 = (dir + 2) % 3; /* velocity roles: cyclic */
  const int a1 = dir == 0 ? 1 : 0, a2 = dir == 2 ? 1 : 2; /* face layout: lower, higher axis */
  int lo[3], hi[3];
  for (int a = 0; a < 3; a++) {
    int act = (a == dir) || swept[a];
    lo[a] = act ? G : 0;
    hi[a] = act ? G + N : M;
  }
  int64_t nfl_total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nfl_total) SERIAL_IF_TAPED
  for (int64_t s = 0; s < m->nleaf; s++) {
    double* B = block_ptr(m, s);
    const double nu = dt / dx_level(m, m->key[4 * s]);
    const int nv = m->nf;
    double* in[6];
    double* fl[6];
    for (int v = 0; v < nv; v++) {
      in[v] = (double*)malloc((size_t)M * sizeof(double));
      fl[v] = (double*)malloc((size_t)M * sizeof(double));
    }
    double* ug = (double*)malloc((size_t)M * sizeof(double));
    const int fmap[6] = {0, 1 + dir, 1 + t1, 1 + t2, 4, 5};
    double* flo = m->face[6 * s + 2 * dir];
    double* fhi = m->face[6 * s + 2 * dir + 1];
    int64_t nfl = 0;
    for (int i2 = lo[t2]; i2 < hi[t2]; i2++)
      for (int i1 = lo[t1]; i1 < hi[t1]; i1++) {
        int pos[3];
        pos[t1] = i1;
        pos[t2] = i2;
        for (int j = 0; j < M; j++) {
          pos[dir] = j;
          for (int v = 0; v < nv; v++) in[v][j] = B[cell(M, fmap[v], pos[0], pos[1], pos[2])];
        }
        pencil(K, nu, M, (const double* const*)in, fl, ug);
        /* flux index k is interface (G-1+k)+1/2 */
        for (int j = G; j < G + N; j++) {
          double Uc[6], Fm[6], Fp[6], Un[6];
          for (int v = 0; v < nv; v++) {
            Uc[v] = in[v][j];
            Fm[v] = fl[v][j - G];
            Fp[v] = fl[v][j - G + 1];
          }
          nfl += update_cell(K, nu, Uc, Fm, Fp, ug[j - G], ug[j - G + 1], Un);
          pos[dir] = j;
          for (int vv = 0; vv < nv; vv++) B[cell(M, fmap[vv], pos[0], pos[1], pos[2])] = Un[vv];
        }
        /* coarse-fine face fluxes, in conserved-field order */
        int ta1 = (a1 == t1) ? i1 : i2, ta2 = (a2 == t1) ? i1 : i2;
        if (ta1 >= G && ta1 < G + N && ta2 >= G && ta2 < G + N) {
          int64_t off = (int64_t)(ta2 - G) * N + (ta1 - G);
          for (int v = 0; v < nv; v++) {
            if (flo) flo[(int64_t)fmap[v] * N * N + off] = fl[v][0];
            if (fhi) fhi[(int64_t)fmap[v] * N * N + off] = fl[v][N];
          }
        }
      }
    nfl_total += nfl;
    for (int v = 0; v < nv; v++) { free(in[v]); free(fl[v]); }
    free(ug);
  }
  m->floors += nfl_total;
}

/* Reflux at coarse-fine faces (Berger & Colella 1989, cited by the paper for
 * AMR): the coarse cell's flux at the face is replaced by the area mean of
 * the 2x2 fine fluxes, F_bar = ((F00 + F10) + (F01 + F11)) * 0.25 (first
 * index along the lower transverse axis), U_c += s nu_c (F_c - F_bar) with
 * s = +1 on the coarse cell's high face and -1 on its low face.  Axes are
 * processed in the order x, y, z. */
static void reflux(orc_mesh* m, double dt) {
  const int N = m->N, M = m->M;
  for (int dir = 0; dir < 3; dir++) {
    const int a1 = dir == 0 ? 1 : 0, a2 = dir == 2 ? 1 : 2;
#pragma omp parallel for schedule(dynamic, 1) SERIAL_IF_TAPED
    for (int64_t s = 0; s < m->nleaf; s++) {
      const int32_t* kk = m->key + 4 * s;
      const int l = kk[0];
      double* B = block_ptr(m, s);
      const double nu = dt / dx_level(m, l);
      for (int side = 0; side < 2; side++) {
        const double* Fc = m->face[6 * s + 2 * dir + side];
        if (!Fc) continue;
        int nb[3] = {kk[1], kk[2], kk[3]};
        nb[dir] += side ? 1 : -1;
        wrap_block(m, l, dir, &nb[dir]);
        if (m->state[l][nidx(m, l, nb[0], nb[1], nb[2])] != REFINED) continue; /* fine side */
        for (int t2 = 0; t2 < N; t2++)
          for (int t1 = 0; t1 < N; t1++) {
            int h1 = t1 >= N / 2, h2 = t2 >= N / 2;
            int cp[3];
            cp[dir] = 2 * nb[dir] + (side ? 0 : 1);
            cp[a1] = 2 * kk[1 + a1] + h1;
            cp[a2] = 2 * kk[1 + a2] + h2;
            int32_t fs = m->leaf_at[l + 1][nidx(m, l + 1, cp[0], cp[1], cp[2])];
            const double* Ff = m->face[6 * (int64_t)fs + 2 * dir + (1 - side)];
            int f1 = 2 * t1 - h1 * N, f2 = 2 * t2 - h2 * N;
            int pos[3];
            pos[dir] = side ? G + N - 1 : G;
            pos[a1] = G + t1;
            pos[a2] = G + t2;
            for (int f = 0; f < m->nf; f++) {
              const double* Q = Ff + (int64_t)f * N * N;
              double fb = ((Q[f2 * N + f1] + Q[f2 * N + f1 + 1]) + (Q[(f2 + 1) * N + f1] + Q[(f2 + 1) * N + f1 + 1])) * 0.25;
              double corr = nu * (Fc[(int64_t)f * N * N + t2 * N + t1] - fb);
              double* u = &B[cell(M, f, pos[0], pos[1], pos[2])];
              *u = side ? *u + corr : *u - corr;
            }
          }
      }
    }
  }
}

void orc_set_debug(int flags) { g_debug = flags; }

void orc_step_dt(orc_mesh* m, int64_t step_index, double dt) {
  const consts_t K = mesh_consts(m);
  orc_refresh(m);
  int order[3] = {0, 1, 2};
  if (step_index & 1) { order[0] = 2; order[2] = 0; }
  int swept[3] = {0, 0, 0};
  for (int s = 0; s < 3; s++) {
    sweep(m, &K, order[s], swept, dt);
    swept[order[s]] = 1;
  }
  if (!(g_debug & ORC_DEBUG_SKIP_REFLUX)) reflux(m, dt);
}

/* Density misfit of the config-4 loss: sum over active leaf cells of
 * (V_c / V_root) (rho_c - target_c)^2, V_c / V_root = 8^-level, summed
 * leaf by leaf, cells z, y, x. */
static double density_misfit(const orc_mesh* m, const double* target) {
  const int N = m->N, M = m->M;
  const int64_t N3 = (int64_t)N * N * N;
  double L = 0.0;
  for (int64_t s = 0; s < m->nleaf; s++) {
    const double* B = block_ptr(m, s);
    const double w = ldexp(1.0, -3 * m->key[4 * s]);
    const double* T = target + s * N3;
    double ls = 0.0;
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) {
          const double d = B[cell(M, 0, a + G, b + G, c + G)] - T[((int64_t)c * N + b) * N + a];
          ls = ls + d * d;
        }
    L = L + w * ls;
  }
  return L;
}

static orc_mesh* clone_mesh(const orc_mesh* m0) {
  orc_mesh* m = NULL;
  if (orc_create_from_leaves(&m0->d, m0->nleaf, m0->key, &m)) return NULL;
  memcpy(m->U, m0->U, (size_t)m0->nleaf * m0->nf * m0->M * m0->M * m0->M * sizeof(double));
  return m;
}

static void run_steps_dt(orc_mesh* m, int64_t first_step, int nsteps, const double* dts) {
  for (int k = 0; k < nsteps; k++) orc_step_dt(m, first_step + k, dts[k]);
}

/* Difference of the misfit between two states a and b of the same mesh,
 * L(a) - L(b) = sum 8^-level (rho_a - rho_b)(rho_a + rho_b - 2 target),
 * written so that L's own size does not cancel. */
static double misfit_difference(const orc_mesh* m, const double* rho_a, const orc_mesh* b, const double* target) {
  const int N = m->N, M = m->M;
  const int64_t N3 = (int64_t)N * N * N;
  double D = 0.0;
  for (int64_t s = 0; s < m->nleaf; s++) {
    const double* B = block_ptr(b, s);
    const double w = ldexp(1.0, -3 * m->key[4 * s]);
    double ds = 0.0;
    for (int c = 0; c < N; c++)
      for (int y = 0; y < N; y++)
        for (int a = 0; a < N; a++) {
          const int64_t q = s * N3 + ((int64_t)c * N + y) * N + a;
          const double ra = rho_a[q], rb = B[cell(M, 0, a + G, y + G, c + G)];
          ds = ds + (ra - rb) * ((ra + rb) - 2.0 * target[q]);
        }
    D = D + w * ds;
  }
  return D;
}

/* A branch tape driven by the caller, for frozen-branch runs of any
 * sequence of oracle calls (comoving steps, say) on the calling thread:
 * orc_tape_record() starts recording the choices of the calls that follow,
 * orc_tape_replay() makes them return the recorded choices from the first,
 * orc_tape_stop() detaches the tape; it returns -1 if the recording ran out
 * of memory or a replay did not consume the recorded choices exactly (the
 * replayed calls were not the recorded ones), else 0. */
static tape_t g_user_tape;
void orc_tape_record(void) {
  free(g_user_tape.b);
  memset(&g_user_tape, 0, sizeof g_user_tape);
  t_tape = &g_user_tape;
}
void orc_tape_replay(void) {
  g_user_tape.pos = 0;
  g_user_tape.replay = 1;
  g_user_tape.overrun = 0;
  t_tape = &g_user_tape;
}
int orc_tape_stop(void) {
  t_tape = NULL;
  if (g_user_tape.overrun || (g_user_tape.replay && g_user_tape.pos != g_user_tape.n))
    return fail("the branch tape was not replayed exactly");
  return 0;
}

int orc_frozen_fd_density_grad(const orc_mesh* m0, int64_t first_step, int nsteps, const double* dts,
                               const double* target, double eps, const int64_t* idx, int64_t nidx,
                               double* grad_out, double* loss_out) {
  if (m0->nf != 5) return fail("frozen-branch differences need a five-field mesh");
  if (nsteps < 0 || !(eps > 0.0)) return fail("nsteps must be >= 0 and eps > 0");
  const int N = m0->N, M = m0->M;
  const int64_t N3 = (int64_t)N * N * N;
  for (int64_t q = 0; q < nidx; q++)
    if (idx[q] < 0 || idx[q] >= m0->nleaf * N3) return fail("density index out of range");
  /* record the base run's choices */
  tape_t rec = {0};
  orc_mesh* base = clone_mesh(m0);
  if (!base) return -1;
  t_tape = &rec;
  run_steps_dt(base, first_step, nsteps, dts);
  t_tape = NULL;
  if (loss_out) *loss_out = density_misfit(base, target);
  orc_destroy(base);
  if (rec.overrun) { free(rec.b); return fail("branch tape allocation failed"); }
  int bad = 0;
#pragma omp parallel reduction(| : bad)
  {
    orc_mesh* m = clone_mesh(m0);
    double* rho_p = (double*)malloc((size_t)(m0->nleaf * N3) * sizeof(double));
    tape_t rep = {rec.b, rec.n, rec.cap, 0, 1, 0};
    if (!m || !rho_p) bad = 1;
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < nidx; q++) {
      if (!m || !rho_p) continue;
      const int64_t s = idx[q] / N3, r = idx[q] - s * N3;
      const int a = (int)(r % N) + G, b = (int)((r / N) % N) + G, c = (int)(r / ((int64_t)N * N)) + G;
      for (int side = 0; side < 2; side++) {
        memcpy(m->U, m0->U, (size_t)m0->nleaf * 5 * M * M * M * sizeof(double));
        double* rho = &block_ptr(m, s)[cell(M, 0, a, b, c)];
        *rho = side ? *rho - eps : *rho + eps;
        rep.pos = 0;
        t_tape = &rep;
        run_steps_dt(m, first_step, nsteps, dts);
        t_tape = NULL;
        if (rep.overrun || rep.pos != rep.n) bad = 1;
        if (side == 0) {
          for (int64_t t = 0; t < m->nleaf; t++)
            for (int cz = 0; cz < N; cz++)
              for (int y = 0; y < N; y++)
                for (int x = 0; x < N; x++)
                  rho_p[t * N3 + ((int64_t)cz * N + y) * N + x] = block_ptr(m, t)[cell(M, 0, x + G, y + G, cz + G)];
        }
      }
      grad_out[q] = misfit_difference(m, rho_p, m, target) / (2.0 * eps);
    }
    if (m) orc_destroy(m);
    free(rho_p);
  }
  free(rec.b);
  return bad ? fail("a replay did not consume the recorded choices exactly") : 0;
}

double orc_step(orc_mesh* m, int64_t step_index) {
  double dt = orc_cfl_dt(m);
  orc_step_dt(m, step_index, dt);
  return dt;
}

/* ------------------------------------------------------------------ */
/* Comoving coordinates (Sec. II-C: the ppm Method with cosmological     */
/* comoving expansion terms, Bryan et al. 1995)                          */
/* ------------------------------------------------------------------ */
/* Readings: x is the comoving position, v the peculiar velocity and a(t)
 * the expansion factor.  The flux divergence carries 1/a, so a step with dt
 * runs the plain sweeps and reflux with the effective dt / a (nu = (dt / a)
 * / dx), and a signal crosses a comoving cell in a dx / (|v| + c): the CFL
 * dt is (C_cfl * a) * min dx / (max_d |v_d| + c).  The expansion sources
 * dv/dt = -H v and d(rho e)/dt = -3 (gamma - 1) H rho e (H = adot / a; rho
 * is the comoving density and does not change) are applied after the reflux
 * with Crank-Nicolson factors at the step's mid time, c = (dt / 2) H:
 * momenta times fv = (1 - c) / (1 + c); internal energy times
 * fe = (1 - 3 (gamma - 1) c) / (1 + 3 (gamma - 1) c); the total energy
 * takes the two changes as E + ((ie' - ie) + ke (fv fv - 1)), so that H = 0
 * leaves the state bit for bit.  Where the source lowered the internal
 * energy below the pressure floor it is raised to it (counted). */

double orc_cfl_dt_comoving(const orc_mesh* m, double a) { return (m->d.cfl * a) * cfl_min(m); }

static void expansion(orc_mesh* m, double dt, double hubble) {
  const consts_t K = mesh_consts(m);
  const int N = m->N, M = m->M;
  const double c = (0.5 * dt) * hubble;
  const double g3 = 3.0 * K.gm1;
  const double fv = (1.0 - c) / (1.0 + c);
  const double fe = (1.0 - g3 * c) / (1.0 + g3 * c);
  int64_t nfl = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nfl) SERIAL_IF_TAPED
  for (int64_t s = 0; s < m->nleaf; s++) {
    double* B = block_ptr(m, s);
    for (int z = G; z < G + N; z++)
      for (int y = G; y < G + N; y++)
        for (int x = G; x < G + N; x++) {
          double* rho = &B[cell(M, 0, x, y, z)];
          double* mx = &B[cell(M, 1, x, y, z)];
          double* my = &B[cell(M, 2, x, y, z)];
          double* mz = &B[cell(M, 3, x, y, z)];
          double* E = &B[cell(M, 4, x, y, z)];
          const double ir = 1.0 / *rho;
          const double u = *mx * ir, v = *my * ir, w = *mz * ir;
          const double ke = (0.5 * *rho) * ((u * u + v * v) + w * w);
          const double ie = *E - ke;
          double ie2 = ie * fe;
          if (BR(ie2 < ie && K.gm1 * ie2 < K.p_floor)) {
            ie2 = (g_debug & ORC_DEBUG_EXP_FLOOR_NO_IG) ? K.p_floor : K.p_floor * K.inv_gm1;
            nfl++;
          }
          *mx = *mx * fv;
          *my = *my * fv;
          *mz = *mz * fv;
          *E = *E + ((ie2 - ie) + ke * (fv * fv - 1.0));
          if (K.de) { /* the dual-energy field takes the same factor and floor rule */
            double* ge = &B[cell(M, 5, x, y, z)];
            double ge2 = *ge * fe;
            if (BR(ge2 < *ge && K.gm1 * ge2 < K.p_floor)) {
              ge2 = K.p_floor * K.inv_gm1;
              nfl++;
            }
            *ge = ge2;
          }
        }
  }
  m->floors += nfl;
}

void orc_step_comoving(orc_mesh* m, int64_t step_index, double dt, double a, double hubble) {
  orc_step_dt(m, step_index, dt / a);
  expansion(m, dt, hubble);
}

/* ------------------------------------------------------------------ */
/* Tracer particles (Sec. II-B: Lagrangian particles live on Blocks and  */
/* move between them; Sec. III: the blast workload carries tracers)      */
/* ------------------------------------------------------------------ */
/* Readings: a position is stored in level-0 cell units, X in [0, Rx*N),
 * so a particle's level-l cell is floor(X * 2^l) (an exact scaling) and
 * wrapping adds or subtracts the integer extent exactly.  A particle belongs
 * to the leaf holding that cell.  The drift uses the velocity of the state at
 * the start of the step with refreshed ghosts: per cell u = m * (1/rho), then
 * trilinear interpolation between the 8 cell centres around the particle,
 * X += (dt * u) * (Rx * N); periodic axes wrap, particles leaving through an
 * outflow face are removed. */

int64_t orc_locate(const orc_mesh* m, const double P[3]) {
  const int N = m->N;
  for (int l = 0; l < m->nlev; l++) {
    int b[3];
    for (int a = 0; a < 3; a++) {
      const double c = floor(ldexp(P[a], l));
      if (!(c >= 0.0)) return -1;
      b[a] = (int)((int64_t)c / N);
      if (b[a] >= m->ext[l][a]) return -1;
    }
    const int64_t q = nidx(m, l, b[0], b[1], b[2]);
    if (m->state[l][q] == LEAF) return m->leaf_at[l][q];
    if (m->state[l][q] != REFINED) return -1;
  }
  return -1;
}

/* Velocity at P inside leaf s (refreshed ghosts), trilinear between the 8
 * surrounding cell centres, summed x, then y, then z. */
static void tracer_velocity(const orc_mesh* m, int64_t s, const double P[3], double v[3]) {
  const int N = m->N, M = m->M;
  const int32_t* kk = m->key + 4 * s;
  const int l = kk[0];
  int i0[3];
  double w[3][2];
  for (int a = 0; a < 3; a++) {
    const double sa = (ldexp(P[a], l) - (double)((int64_t)kk[1 + a] * N)) - 0.5;
    const double fl = floor(sa);
    i0[a] = (int)fl + G;
    const double f = sa - fl;
    w[a][0] = 1.0 - f;
    w[a][1] = f;
  }
  const double* B = block_ptr(m, s);
  double c[3][2][2][2];  /* component, dz, dy, dx */
  for (int dz = 0; dz < 2; dz++)
    for (int dy = 0; dy < 2; dy++)
      for (int dx = 0; dx < 2; dx++) {
        const int a = i0[0] + dx, b = i0[1] + dy, cc = i0[2] + dz;
        const double ir = 1.0 / B[cell(M, 0, a, b, cc)];
        for (int d = 0; d < 3; d++) c[d][dz][dy][dx] = B[cell(M, 1 + d, a, b, cc)] * ir;
      }
  for (int d = 0; d < 3; d++) {
    const double z0 = (c[d][0][0][0] * w[0][0] + c[d][0][0][1] * w[0][1]) * w[1][0] +
                      (c[d][0][1][0] * w[0][0] + c[d][0][1][1] * w[0][1]) * w[1][1];
    const double z1 = (c[d][1][0][0] * w[0][0] + c[d][1][0][1] * w[0][1]) * w[1][0] +
                      (c[d][1][1][0] * w[0][0] + c[d][1][1][1] * w[0][1]) * w[1][1];
    v[d] = z0 * w[2][0] + z1 * w[2][1];
  }
}

int64_t orc_tracers_drift(const orc_mesh* m, double dt, int64_t n, double* X, double* Y, double* Z,
                          int32_t* alive) {
  const double n0 = (double)((int64_t)m->d.root[0] * m->N);
  int64_t removed = 0;
#pragma omp parallel for reduction(+ : removed) schedule(static)
  for (int64_t i = 0; i < n; i++) {
    if (!alive[i]) continue;
    double P[3] = {X[i], Y[i], Z[i]};
    const int64_t s = orc_locate(m, P);
    if (s < 0) { alive[i] = 0; removed++; continue; }
    double v[3];
    tracer_velocity(m, s, P, v);
    int out = 0;
    for (int a = 0; a < 3; a++) {
      const double E = (double)((int64_t)m->d.root[a] * m->N);
      double x = P[a] + (dt * v[a]) * n0;
      if (m->d.bc[a] == ORC_BC_PERIODIC) {
        if (x < 0.0) x += E;
        if (x >= E) x -= E;
      } else if (x < 0.0 || x >= E) {
        out = 1;
      }
      P[a] = x;
    }
    if (out) { alive[i] = 0; removed++; continue; }
    X[i] = P[0]; Y[i] = P[1]; Z[i] = P[2];
  }
  return removed;
}

double orc_step_tracers(orc_mesh* m, int64_t step_index, int64_t n, double* X, double* Y, double* Z,
                        int32_t* alive) {
  const double dt = orc_cfl_dt(m);
  orc_refresh(m);
  orc_tracers_drift(m, dt, n, X, Y, Z, alive);
  orc_step_dt(m, step_index, dt);  /* refreshes again: the same ghosts */
  return dt;
}

/* ------------------------------------------------------------------ */
/* mg0 on the octree (Sec. II-C: the gravity Method's multigrid solver;  */
/* Sec. II-B: the array of octrees it runs on)                           */
/* ------------------------------------------------------------------ */
/* Readings (the paper names mg0 and the octree, not the discretisation):
 *  - unknowns: one value per active leaf cell.  The operator is the
 *    finite-volume Laplacian -- per cell, the sum over its 6 faces of the
 *    outward difference quotient, divided by h -- written as the 7-point sum
 *    on ghost-filled blocks plus a correction at coarse-fine faces:
 *    L = (S - 6 phi) (1/h^2), S = ((W + E) + (S + N)) + (B + T) from the
 *    block's ghosts, which hold same-level copies, the mean of the 8
 *    children over finer leaves, and over a coarser leaf its linear
 *    interpolation with central slopes,
 *    g = ((phi_P + 0.25 o_x s_x) + 0.25 o_y s_y) + 0.25 o_z s_z,
 *    s_d = 0.5 (phi_{P+e_d} - phi_{P-e_d});
 *    at a coarse cell's face onto finer leaves the coarse quotient
 *    F_c = (g_c - phi_c) (1/h) (g_c the restricted ghost) is replaced by the
 *    mean of the four fine cells' quotients across that face, taken outward
 *    from the coarse cell, F_k = (phi_k - g_k) (1/h_f):
 *    L += ((((F00 + F10) + (F01 + F11)) 0.25) - F_c) (1/h), axes x, y, z in
 *    turn (first index along the lower transverse axis).  The fluxes through
 *    a coarse-fine face then agree on both sides, so the volume-weighted sum
 *    of L phi over a periodic mesh vanishes.
 *  - hierarchy: Omega_l = the leaves coarser than l and every octree node of
 *    level l, for l = L_max (the mesh itself) down to 1, then Omega_0 = the
 *    root blocks, a uniform periodic grid.
 *  - V-cycle on Omega_l (l >= 1; correction form): nu1 red-black passes, the
 *    residual, its restriction to Omega_{l-1} (a level-(l-1) node's cell is
 *    the mean of its 8 children's residuals, summed as the refresh's
 *    restriction; unchanged cells copy), the correction on Omega_{l-1} from
 *    zero, then added back: the copy on unchanged cells, on a level-l cell
 *    the interpolation formula above from its parent (correction ghosts
 *    refreshed the same way), then nu2 red-black passes.  On Omega_0: one
 *    uniform mg0 V-cycle from zero (the uniform solver's own levels below).
 *  - red-black pass of colour c ((i + j + k) even first, global indices at
 *    the cell's level): refresh, then for every leaf cell of colour c,
 *    r = f - L phi from the values before the pass, then phi -= r / D,
 *    D = (6 + n_cf) (1/h^2) (minus L's diagonal coefficient), n_cf = the
 *    cell's coarse-side coarse-fine faces (each such face doubles its
 *    diagonal coefficient).
 *  - a solve: f minus its volume-weighted mean; ncycles V-cycles from the
 *    caller's phi; phi minus its volume-weighted mean.  A cell weighs 8^-level;
 *    sums run leaf by leaf, cells z, y, x.  An unrefined mesh takes the
 *    uniform solver's path exactly. */

static int g_mgc_debug = 0;
void orc_mgc_set_debug(int flags) { g_mgc_debug = flags; }

typedef struct {
  const orc_mesh* m;
  orc_mesh* own;
  double* x; /* nleaf x M^3, ghost-filled on use */
  double* b; /* nleaf x N^3 */
  double* L; /* nleaf x N^3 */
  unsigned char* ncf; /* nleaf x N^3 */
} mgc_stage;

static inline int64_t acell(int N, int64_t s, int a, int b, int c) {
  return (s * N + c) * (int64_t)N * N + (int64_t)b * N + a;
}

static void mgc_refresh(const orc_mesh* m, double* x) {
  const int lin = (g_mgc_debug & ORC_MGC_DEBUG_FLAT) ? 2 : 1;
  refresh_fields(m, x, 1, 1, lin);
  refresh_fields(m, x, 1, 2, lin);
}

/* L phi (and the coarse-side coarse-fine face counts) on the cells of
 * colour col (-1: all), from the ghost-filled x. */
static void mgc_lap(const orc_mesh* m, const double* x, double* Lout, unsigned char* ncf, int col) {
  const int N = m->N, M = m->M;
  const int64_t M3 = (int64_t)M * M * M;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < m->nleaf; s++) {
    const int32_t* kk = m->key + 4 * s;
    const int l = kk[0];
    const double h = dx_level(m, l), ih = 1.0 / h, ih2 = 1.0 / (h * h);
    const double ihf = 1.0 / dx_level(m, l + 1);
    const double* X = x + s * M3;
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) {
          if (col >= 0 && ((a + b + c) & 1) != col) continue;
          const int A = a + G, B = b + G, C = c + G;
          const double xc = X[cell(M, 0, A, B, C)];
          const double S = ((X[cell(M, 0, A - 1, B, C)] + X[cell(M, 0, A + 1, B, C)]) +
                            (X[cell(M, 0, A, B - 1, C)] + X[cell(M, 0, A, B + 1, C)])) +
                           (X[cell(M, 0, A, B, C - 1)] + X[cell(M, 0, A, B, C + 1)]);
          double L = (S - 6.0 * xc) * ih2;
          int n = 0;
          const int loc[3] = {a, b, c};
          for (int dir = 0; dir < 3 && !(g_mgc_debug & ORC_MGC_DEBUG_NO_MATCH); dir++) {
            const int side = loc[dir] == 0 ? 0 : (loc[dir] == N - 1 ? 1 : -1);
            if (side < 0) continue;
            int nb[3] = {kk[1], kk[2], kk[3]};
            nb[dir] += side ? 1 : -1;
            if (!wrap_block(m, l, dir, &nb[dir])) continue;
            if (m->state[l][nidx(m, l, nb[0], nb[1], nb[2])] != REFINED) continue;
            const int a1 = dir == 0 ? 1 : 0, a2 = dir == 2 ? 1 : 2;
            int gp[3] = {A, B, C};
            gp[dir] += side ? 1 : -1;
            const double Fc = (X[cell(M, 0, gp[0], gp[1], gp[2])] - xc) * ih;
            /* the four fine cells across the face, global level-(l+1) indices */
            const int64_t P[3] = {(int64_t)kk[1] * N + a, (int64_t)kk[2] * N + b, (int64_t)kk[3] * N + c};
            double F[2][2];
            for (int q2 = 0; q2 < 2; q2++)
              for (int q1 = 0; q1 < 2; q1++) {
                int64_t fq[3];
                fq[dir] = side ? 2 * P[dir] + 2 : 2 * P[dir] - 1;
                fq[a1] = 2 * P[a1] + q1;
                fq[a2] = 2 * P[a2] + q2;
                for (int ax = 0; ax < 3; ax++) fq[ax] = bc_cell(m, l + 1, ax, fq[ax]);
                const int fb[3] = {(int)(fq[0] / N), (int)(fq[1] / N), (int)(fq[2] / N)};
                const int32_t fs = m->leaf_at[l + 1][nidx(m, l + 1, fb[0], fb[1], fb[2])];
                const double* XF = x + fs * M3;
                int fl[3];
                for (int ax = 0; ax < 3; ax++) fl[ax] = (int)(fq[ax] - (int64_t)fb[ax] * N) + G;
                const double xf = XF[cell(M, 0, fl[0], fl[1], fl[2])];
                fl[dir] += side ? -1 : 1; /* the fine cell's ghost inside the coarse cell */
                const double gf = XF[cell(M, 0, fl[0], fl[1], fl[2])];
                F[q1][q2] = (xf - gf) * ihf;
              }
            const double Fbar = ((F[0][0] + F[1][0]) + (F[0][1] + F[1][1])) * 0.25;
            L = L + (Fbar - Fc) * ih;
            n++;
          }
          Lout[acell(N, s, a, b, c)] = L;
          if (ncf) ncf[acell(N, s, a, b, c)] = (unsigned char)n;
        }
  }
}

static void mgc_pass(mgc_stage* st, int col) {
  const orc_mesh* m = st->m;
  const int N = m->N, M = m->M;
  const int64_t M3 = (int64_t)M * M * M;
  mgc_refresh(m, st->x);
  mgc_lap(m, st->x, st->L, st->ncf, col);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < m->nleaf; s++) {
    const double h = dx_level(m, m->key[4 * s]), ih2 = 1.0 / (h * h);
    double* X = st->x + s * M3;
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) {
          if (((a + b + c) & 1) != col) continue;
          const int64_t q = acell(N, s, a, b, c);
          const double r = st->b[q] - st->L[q];
          const double D = (double)(6 + st->ncf[q]) * ih2;
          double* xc = &X[cell(M, 0, a + G, b + G, c + G)];
          *xc = *xc - r / D;
        }
  }
}

/* r = f - L phi on every cell into st->L (overwritten). */
static void mgc_residual(mgc_stage* st) {
  const int64_t n = st->m->nleaf * (int64_t)st->m->N * st->m->N * st->m->N;
  mgc_refresh(st->m, st->x);
  mgc_lap(st->m, st->x, st->L, NULL, -1);
  for (int64_t q = 0; q < n; q++) st->L[q] = st->b[q] - st->L[q];
}

static int32_t leaf_of(const orc_mesh* m, int l, int i, int j, int k) {
  if (l >= m->nlev) return -1;
  const int64_t q = nidx(m, l, i, j, k);
  return m->state[l][q] == LEAF ? m->leaf_at[l][q] : -1;
}

/* Omega_l's residual (in F->L) restricted into C->b (Omega_{l-1}). */
static void mgc_restrict(const mgc_stage* F, mgc_stage* C) {
  const orc_mesh* fm = F->m;
  const orc_mesh* cm = C->m;
  const int N = cm->N;
  for (int64_t t = 0; t < cm->nleaf; t++) {
    const int32_t* kk = cm->key + 4 * t;
    const int32_t same = leaf_of(fm, kk[0], kk[1], kk[2], kk[3]);
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) {
          double v;
          if (same >= 0) {
            v = F->L[acell(N, same, a, b, c)];
          } else {
            double w8[8];
            for (int o = 0; o < 8; o++) {
              const int fa = 2 * a + (o & 1), fb = 2 * b + ((o >> 1) & 1), fc = 2 * c + (o >> 2);
              const int32_t fs = leaf_of(fm, kk[0] + 1, 2 * kk[1] + fa / N, 2 * kk[2] + fb / N, 2 * kk[3] + fc / N);
              w8[o] = F->L[acell(N, fs, fa % N, fb % N, fc % N)];
            }
            v = restrict8(w8);
          }
          C->b[acell(N, t, a, b, c)] = v;
        }
  }
}

/* Omega_l's x += the interpolation of Omega_{l-1}'s correction (C->x,
 * refreshed here). */
static void mgc_prolong_add(mgc_stage* C, mgc_stage* F) {
  const orc_mesh* cm = C->m;
  const orc_mesh* fm = F->m;
  const int N = fm->N, M = fm->M;
  const int64_t M3 = (int64_t)M * M * M;
  mgc_refresh(cm, C->x);
  for (int64_t s = 0; s < fm->nleaf; s++) {
    const int32_t* kk = fm->key + 4 * s;
    double* X = F->x + s * M3;
    const int32_t same = leaf_of(cm, kk[0], kk[1], kk[2], kk[3]);
    const int32_t par = same >= 0 ? -1 : leaf_of(cm, kk[0] - 1, kk[1] >> 1, kk[2] >> 1, kk[3] >> 1);
    const double* E = C->x + (same >= 0 ? same : par) * M3;
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) {
          double v;
          if (same >= 0) {
            v = E[cell(M, 0, a + G, b + G, c + G)];
          } else {
            const int g[3] = {(kk[1] & 1) * N + a, (kk[2] & 1) * N + b, (kk[3] & 1) * N + c};
            const int lc[3] = {g[0] / 2 + G, g[1] / 2 + G, g[2] / 2 + G};
            double o[3], sl[3];
            for (int ax = 0; ax < 3; ax++) o[ax] = (g[ax] & 1) ? 1.0 : -1.0;
            const double u0 = E[cell(M, 0, lc[0], lc[1], lc[2])];
            if (g_mgc_debug & ORC_MGC_DEBUG_FLAT) {
              sl[0] = sl[1] = sl[2] = 0.0;
            } else {
              sl[0] = 0.5 * (E[cell(M, 0, lc[0] + 1, lc[1], lc[2])] - E[cell(M, 0, lc[0] - 1, lc[1], lc[2])]);
              sl[1] = 0.5 * (E[cell(M, 0, lc[0], lc[1] + 1, lc[2])] - E[cell(M, 0, lc[0], lc[1] - 1, lc[2])]);
              sl[2] = 0.5 * (E[cell(M, 0, lc[0], lc[1], lc[2] + 1)] - E[cell(M, 0, lc[0], lc[1], lc[2] - 1)]);
            }
            v = ((u0 + (0.25 * o[0]) * sl[0]) + (0.25 * o[1]) * sl[1]) + (0.25 * o[2]) * sl[2];
          }
          double* xc = &X[cell(M, 0, a + G, b + G, c + G)];
          *xc = *xc + v;
        }
  }
}

/* Block storage (per leaf N^3 at level 0) <-> the global root grid. */
static void root_gather(const orc_mesh* m, const double* blocks, int64_t stride, int off, double* g) {
  const int N = m->N, n0 = m->d.root[0] * N, n1 = m->d.root[1] * N;
  for (int64_t s = 0; s < m->nleaf; s++) {
    const int32_t* kk = m->key + 4 * s;
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) {
          const int64_t q = stride ? s * stride + cell(m->M, 0, a + off, b + off, c + off) : acell(N, s, a, b, c);
          g[((int64_t)(kk[3] * N + c) * n1 + (kk[2] * N + b)) * n0 + (kk[1] * N + a)] = blocks[q];
        }
  }
}
static void root_scatter(const orc_mesh* m, const double* g, double* blocks, int64_t stride, int off) {
  const int N = m->N, n0 = m->d.root[0] * N, n1 = m->d.root[1] * N;
  for (int64_t s = 0; s < m->nleaf; s++) {
    const int32_t* kk = m->key + 4 * s;
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) {
          const int64_t q = stride ? s * stride + cell(m->M, 0, a + off, b + off, c + off) : acell(N, s, a, b, c);
          blocks[q] = g[((int64_t)(kk[3] * N + c) * n1 + (kk[2] * N + b)) * n0 + (kk[1] * N + a)];
        }
  }
}

static void mgc_vcycle(mgc_stage* st, int l, int nu1, int nu2) {
  mgc_stage* S = &st[l];
  const orc_mesh* m = S->m;
  const int N = m->N, M = m->M;
  if (l == 0) {
    const int n[3] = {m->d.root[0] * N, m->d.root[1] * N, m->d.root[2] * N};
    const int64_t cnt = (int64_t)n[0] * n[1] * n[2];
    double* f = (double*)malloc((size_t)cnt * sizeof(double));
    double* e = (double*)malloc((size_t)cnt * sizeof(double));
    root_gather(m, S->b, 0, 0, f);
    orc_mg_vcycle_from_zero(n[0], n[1], n[2], dx_level(m, 0), f, e, nu1, nu2);
    memset(S->x, 0, (size_t)m->nleaf * M * M * M * sizeof(double));
    root_scatter(m, e, S->x, (int64_t)M * M * M, G);
    free(f);
    free(e);
    return;
  }
  for (int k = 0; k < nu1; k++) {
    mgc_pass(S, 0);
    mgc_pass(S, 1);
  }
  mgc_residual(S);
  mgc_restrict(S, &st[l - 1]);
  /* the correction on the coarser hierarchy level starts from zero */
  memset(st[l - 1].x, 0, (size_t)st[l - 1].m->nleaf * M * M * M * sizeof(double));
  mgc_vcycle(st, l - 1, nu1, nu2);
  mgc_prolong_add(&st[l - 1], S);
  for (int k = 0; k < nu2; k++) {
    mgc_pass(S, 0);
    mgc_pass(S, 1);
  }
}

static double weighted_sum(const orc_mesh* m, const double* v, int sq, double* vol) {
  const int64_t N3 = (int64_t)m->N * m->N * m->N;
  double tot = 0.0, vv = 0.0;
  for (int64_t s = 0; s < m->nleaf; s++) {
    const double w = ldexp(1.0, -3 * m->key[4 * s]);
    double ls = 0.0;
    for (int64_t q = 0; q < N3; q++) ls = ls + (sq ? v[s * N3 + q] * v[s * N3 + q] : v[s * N3 + q]);
    tot = tot + w * ls;
    vv = vv + w * (double)N3;
  }
  if (vol) *vol = vv;
  return tot;
}

int orc_mgc_apply(const orc_mesh* m, const double* phi, double* out) {
  for (int a = 0; a < 3; a++)
    if (m->d.bc[a] != ORC_BC_PERIODIC) return fail("mg0 on the octree needs periodic boundaries");
  const int N = m->N, M = m->M;
  double* x = (double*)calloc((size_t)m->nleaf * M * M * M, sizeof(double));
  for (int64_t s = 0; s < m->nleaf; s++)
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) x[s * (int64_t)M * M * M + cell(M, 0, a + G, b + G, c + G)] = phi[acell(N, s, a, b, c)];
  mgc_refresh(m, x);
  mgc_lap(m, x, out, NULL, -1);
  free(x);
  return 0;
}

int orc_mgc_solve(const orc_mesh* m, const double* f, double* phi, int ncycles, int nu1, int nu2, double* resid) {
  const int N = m->N, M = m->M;
  const int64_t M3 = (int64_t)M * M * M, N3 = (int64_t)N * N * N;
  int n[3];
  for (int a = 0; a < 3; a++) {
    if (m->d.bc[a] != ORC_BC_PERIODIC) return fail("mg0 on the octree needs periodic boundaries");
    n[a] = m->d.root[a] * N;
  }
  if (ncycles < 0 || nu1 < 0 || nu2 < 0) return fail("ncycles, nu1 and nu2 must be >= 0");
  int lmax = 0;
  for (int64_t s = 0; s < m->nleaf; s++) lmax = m->key[4 * s] > lmax ? m->key[4 * s] : lmax;
  if (lmax == 0) {
    /* the uniform solver exactly */
    const int64_t cnt = (int64_t)n[0] * n[1] * n[2];
    double* fg = (double*)malloc((size_t)cnt * sizeof(double));
    double* pg = (double*)malloc((size_t)cnt * sizeof(double));
    root_gather(m, f, 0, 0, fg);
    root_gather(m, phi, 0, 0, pg);
    const int nl = orc_mg_solve(n[0], n[1], n[2], dx_level(m, 0), fg, pg, ncycles, nu1, nu2, resid);
    root_scatter(m, pg, phi, 0, 0);
    free(fg);
    free(pg);
    return nl;
  }
  mgc_stage st[ORC_MAXLEV];
  memset(st, 0, sizeof st);
  int rc = 0;
  for (int l = lmax; l >= 0 && !rc; l--) {
    if (l == lmax) {
      st[l].m = m;
    } else {
      /* leaves coarser than l and every node of level l */
      int64_t cnt = 0;
      for (int64_t s = 0; s < m->nleaf; s++) cnt += m->key[4 * s] < l;
      const int64_t nl = (int64_t)m->ext[l][0] * m->ext[l][1] * m->ext[l][2];
      int32_t* keys = (int32_t*)malloc((size_t)(cnt + nl) * 4 * sizeof(int32_t));
      int64_t k = 0;
      for (int64_t s = 0; s < m->nleaf; s++)
        if (m->key[4 * s] < l) memcpy(keys + 4 * k++, m->key + 4 * s, 4 * sizeof(int32_t));
      for (int kz = 0; kz < m->ext[l][2]; kz++)
        for (int ky = 0; ky < m->ext[l][1]; ky++)
          for (int kx = 0; kx < m->ext[l][0]; kx++)
            if (m->state[l][nidx(m, l, kx, ky, kz)] != ABSENT) {
              int32_t* e = keys + 4 * k++;
              e[0] = l; e[1] = kx; e[2] = ky; e[3] = kz;
            }
      rc = orc_create_from_leaves(&m->d, k, keys, &st[l].own);
      free(keys);
      st[l].m = st[l].own;
    }
    if (rc) break;
    const int64_t nb = st[l].m->nleaf;
    st[l].x = (double*)calloc((size_t)(nb * M3), sizeof(double));
    st[l].b = (double*)calloc((size_t)(nb * N3), sizeof(double));
    st[l].L = (double*)calloc((size_t)(nb * N3), sizeof(double));
    st[l].ncf = (unsigned char*)calloc((size_t)(nb * N3), 1);
  }
  int nlev = -1;
  if (!rc) {
    mgc_stage* T = &st[lmax];
    double vol;
    const double fm = weighted_sum(m, f, 0, &vol) / vol;
    for (int64_t q = 0; q < m->nleaf * N3; q++) T->b[q] = f[q] - fm;
    for (int64_t s = 0; s < m->nleaf; s++)
      for (int c = 0; c < N; c++)
        for (int b = 0; b < N; b++)
          for (int a = 0; a < N; a++) T->x[s * M3 + cell(M, 0, a + G, b + G, c + G)] = phi[acell(N, s, a, b, c)];
    if (resid) {
      mgc_residual(T);
      resid[0] = sqrt(weighted_sum(m, T->L, 1, NULL));
    }
    for (int cyc = 0; cyc < ncycles; cyc++) {
      mgc_vcycle(st, lmax, nu1, nu2);
      if (resid) {
        mgc_residual(T);
        resid[cyc + 1] = sqrt(weighted_sum(m, T->L, 1, NULL));
      }
    }
    for (int64_t s = 0; s < m->nleaf; s++)
      for (int c = 0; c < N; c++)
        for (int b = 0; b < N; b++)
          for (int a = 0; a < N; a++) T->L[acell(N, s, a, b, c)] = T->x[s * M3 + cell(M, 0, a + G, b + G, c + G)];
    const double pm = weighted_sum(m, T->L, 0, &vol) / vol;
    for (int64_t q = 0; q < m->nleaf * N3; q++) phi[q] = T->L[q] - pm;
    nlev = lmax + orc_mg_levels(n[0], n[1], n[2]);
  }
  for (int l = 0; l <= lmax; l++) {
    if (st[l].own) orc_destroy(st[l].own);
    free(st[l].x);
    free(st[l].b);
    free(st[l].L);
    free(st[l].ncf);
  }
  return rc ? -1 : nlev;
}

/* ------------------------------------------------------------------ */
/* Self-gravity on a uniform mesh (Sec. II-C: the gravity Method with    */
/* the mg0 solver; Sec. III: self-gravity on a uniform mesh)             */
/* ------------------------------------------------------------------ */
/* Readings: the potential solves lap(phi) = 4 pi G (rho - mean rho) with
 * mg0 on the level-0 grid (warm-started from the caller's phi); the
 * acceleration is g = -grad(phi) by central differences, g_a = (phi(a-1) -
 * phi(a+1)) (1 / (2 dx)); a step is kick-drift-kick: a half kick with the
 * start-of-step phi, the hydro step (dt from the CFL condition), phi from
 * the new density, a half kick with it.  A kick changes the momentum by
 * (dt/2) rho g and the total energy by the change of the kinetic energy
 * (ke = (0.5 rho)((ux ux + uy uy) + uz uz), u = m (1/rho)), so it leaves the
 * internal energy (and rho e) unchanged; G = 0 leaves every bit unchanged. */

static int gravity_grid(const orc_mesh* m, int n[3]) {
  for (int64_t s = 0; s < m->nleaf; s++)
    if (m->key[4 * s] != 0) return fail("self-gravity needs a uniform mesh");
  for (int a = 0; a < 3; a++) {
    if (m->d.bc[a] != ORC_BC_PERIODIC) return fail("self-gravity needs periodic boundaries");
    n[a] = m->d.root[a] * m->N;
  }
  return 0;
}

static void density_source(const orc_mesh* m, const int n[3], double four_pi_G, double* f) {
  const int N = m->N, M = m->M;
  for (int64_t s = 0; s < m->nleaf; s++) {
    const double* B = block_ptr(m, s);
    const int32_t* kk = m->key + 4 * s;
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) {
          const int64_t g = ((int64_t)(kk[3] * N + c) * n[1] + (kk[2] * N + b)) * n[0] + (kk[1] * N + a);
          f[g] = four_pi_G * B[cell(M, 0, a + G, b + G, c + G)];
        }
  }
}

static void kick(orc_mesh* m, const int n[3], const double* phi, double hdt) {
  const int N = m->N, M = m->M;
  const double inv2h = 1.0 / (2.0 * dx_level(m, 0));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < m->nleaf; s++) {
    double* B = block_ptr(m, s);
    const int32_t* kk = m->key + 4 * s;
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) {
          const int p[3] = {kk[1] * N + a, kk[2] * N + b, kk[3] * N + c};
          double gv[3];
          for (int ax = 0; ax < 3; ax++) {
            int lo[3] = {p[0], p[1], p[2]}, hi[3] = {p[0], p[1], p[2]};
            lo[ax] = (p[ax] + n[ax] - 1) % n[ax];
            hi[ax] = (p[ax] + 1) % n[ax];
            const double pl = phi[((int64_t)lo[2] * n[1] + lo[1]) * n[0] + lo[0]];
            const double ph = phi[((int64_t)hi[2] * n[1] + hi[1]) * n[0] + hi[0]];
            gv[ax] = (pl - ph) * inv2h;
          }
          double* rho = &B[cell(M, 0, a + G, b + G, c + G)];
          double* mom[3] = {&B[cell(M, 1, a + G, b + G, c + G)], &B[cell(M, 2, a + G, b + G, c + G)],
                            &B[cell(M, 3, a + G, b + G, c + G)]};
          double* E = &B[cell(M, 4, a + G, b + G, c + G)];
          const double ir = 1.0 / *rho;
          double u[3], u2[3];
          for (int ax = 0; ax < 3; ax++) u[ax] = *mom[ax] * ir;
          const double ke = (0.5 * *rho) * ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
          for (int ax = 0; ax < 3; ax++) {
            const double g = (g_debug & ORC_DEBUG_GRAVITY_SIGN) ? -gv[ax] : gv[ax];
            *mom[ax] = *mom[ax] + hdt * (*rho * g);
            u2[ax] = *mom[ax] * ir;
          }
          const double ke2 = (0.5 * *rho) * ((u2[0] * u2[0] + u2[1] * u2[1]) + u2[2] * u2[2]);
          *E = *E + (ke2 - ke);
        }
  }
}

/* Self-gravity on a refined mesh (mg0 on the octree): the same
 * kick-drift-kick with phi on the leaves (per leaf N^3), solved by the
 * composite V-cycles; g = -grad(phi) by central differences at each cell's
 * own level, g_a = (phi(a-1) - phi(a+1)) (1 / (2 dx_l)), the neighbours
 * across a block face taken from the composite operator's ghosts (copies,
 * 8-child means, linear interpolation from a coarser leaf).  On an
 * unrefined mesh this is orc_step_gravity bit for bit. */
static void density_blocks(const orc_mesh* m, double four_pi_G, double* f) {
  const int N = m->N, M = m->M;
  for (int64_t s = 0; s < m->nleaf; s++) {
    const double* B = block_ptr(m, s);
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) f[acell(N, s, a, b, c)] = four_pi_G * B[cell(M, 0, a + G, b + G, c + G)];
  }
}

static void kick_blocks(orc_mesh* m, const double* phi, double hdt) {
  const int N = m->N, M = m->M;
  const int64_t M3 = (int64_t)M * M * M;
  double* x = (double*)calloc((size_t)(m->nleaf * M3), sizeof(double));
  for (int64_t s = 0; s < m->nleaf; s++)
    for (int c = 0; c < N; c++)
      for (int b = 0; b < N; b++)
        for (int a = 0; a < N; a++) x[s * M3 + cell(M, 0, a + G, b + G, c + G)] = phi[acell(N, s, a, b, c)];
  mgc_refresh(m, x);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < m->nleaf; s++) {
    double* B = block_ptr(m, s);
    const double* X = x + s * M3;
    const double inv2h = 1.0 / (2.0 * dx_level(m, m->key[4 * s]));
    for (int c = G; c < G + N; c++)
      for (int b = G; b < G + N; b++)
        for (int a = G; a < G + N; a++) {
          const int lo[3][3] = {{a - 1, b, c}, {a, b - 1, c}, {a, b, c - 1}};
          const int hi[3][3] = {{a + 1, b, c}, {a, b + 1, c}, {a, b, c + 1}};
          double gv[3];
          for (int ax = 0; ax < 3; ax++)
            gv[ax] = (X[cell(M, 0, lo[ax][0], lo[ax][1], lo[ax][2])] - X[cell(M, 0, hi[ax][0], hi[ax][1], hi[ax][2])]) *
                     inv2h;
          double* rho = &B[cell(M, 0, a, b, c)];
          double* mom[3] = {&B[cell(M, 1, a, b, c)], &B[cell(M, 2, a, b, c)], &B[cell(M, 3, a, b, c)]};
          double* E = &B[cell(M, 4, a, b, c)];
          const double ir = 1.0 / *rho;
          double u[3], u2[3];
          for (int ax = 0; ax < 3; ax++) u[ax] = *mom[ax] * ir;
          const double ke = (0.5 * *rho) * ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
          for (int ax = 0; ax < 3; ax++) {
            const double g = (g_debug & ORC_DEBUG_GRAVITY_SIGN) ? -gv[ax] : gv[ax];
            *mom[ax] = *mom[ax] + hdt * (*rho * g);
            u2[ax] = *mom[ax] * ir;
          }
          const double ke2 = (0.5 * *rho) * ((u2[0] * u2[0] + u2[1] * u2[1]) + u2[2] * u2[2]);
          *E = *E + (ke2 - ke);
        }
  }
  free(x);
}

double orc_step_gravity_amr(orc_mesh* m, int64_t step_index, double four_pi_G, double* phi, int phi_current,
                            int ncycles, int nu1, int nu2) {
  for (int a = 0; a < 3; a++)
    if (m->d.bc[a] != ORC_BC_PERIODIC) return (fail("self-gravity needs periodic boundaries"), -1.0);
  const int64_t n = m->nleaf * (int64_t)m->N * m->N * m->N;
  double* f = (double*)malloc((size_t)n * sizeof(double));
  if (!phi_current) {
    density_blocks(m, four_pi_G, f);
    if (orc_mgc_solve(m, f, phi, ncycles, nu1, nu2, NULL) < 0) { free(f); return -1.0; }
  }
  const double dt = orc_cfl_dt(m);
  kick_blocks(m, phi, 0.5 * dt);
  orc_step_dt(m, step_index, dt);
  density_blocks(m, four_pi_G, f);
  orc_mgc_solve(m, f, phi, ncycles, nu1, nu2, NULL);
  kick_blocks(m, phi, 0.5 * dt);
  free(f);
  return dt;
}

double orc_step_gravity(orc_mesh* m, int64_t step_index, double four_pi_G, double* phi, int phi_current,
                        int ncycles, int nu1, int nu2) {
  int n[3];
  if (gravity_grid(m, n) != 0) return -1.0;
  const double h = dx_level(m, 0);
  double* f = (double*)malloc((size_t)n[0] * n[1] * n[2] * sizeof(double));
  if (!phi_current) {
    density_source(m, n, four_pi_G, f);
    orc_mg_solve(n[0], n[1], n[2], h, f, phi, ncycles, nu1, nu2, NULL);
  }
  const double dt = orc_cfl_dt(m);
  kick(m, n, phi, 0.5 * dt);
  orc_step_dt(m, step_index, dt);
  density_source(m, n, four_pi_G, f);
  orc_mg_solve(n[0], n[1], n[2], h, f, phi, ncycles, nu1, nu2, NULL);
  kick(m, n, phi, 0.5 * dt);
  free(f);
  return dt;
}

/* Comoving self-gravity (Bryan et al. 1995): with the comoving density the
 * momentum source is -(rho / a^2) grad(phi), phi solving lap(phi) =
 * 4 pi G (rho - mean rho) (free of a, so a potential carried from one step
 * to the next stays exact).  A step with the caller's dt (the comoving CFL
 * dt), a at its start, middle and end and H at its middle: a half kick with
 * (dt/2) / a0^2, the expansion sources over dt/2, the hydro step with
 * dt / a_mid, the expansion sources over dt/2 (both halves with H; the
 * symmetric split keeps the step second order, where sources after the
 * drift made the growth of a perturbation first order in dt), phi of the
 * new density, a half kick with (dt/2) / a1^2.  With a = 1 everywhere and
 * H = 0 it is the plain self-gravity step with that dt. */
int orc_step_gravity_comoving(orc_mesh* m, int64_t step_index, double dt, double a0, double a_mid, double a1,
                              double hubble, double four_pi_G, double* phi, int phi_current, int ncycles, int nu1,
                              int nu2) {
  int n[3];
  if (gravity_grid(m, n) != 0) return -1;
  const double h = dx_level(m, 0);
  const int no_a = (g_debug & ORC_DEBUG_GRAVITY_NO_A) != 0;
  const double s0 = no_a ? 1.0 : 1.0 / (a0 * a0), s1 = no_a ? 1.0 : 1.0 / (a1 * a1);
  double* f = (double*)malloc((size_t)n[0] * n[1] * n[2] * sizeof(double));
  if (!phi_current) {
    density_source(m, n, four_pi_G, f);
    orc_mg_solve(n[0], n[1], n[2], h, f, phi, ncycles, nu1, nu2, NULL);
  }
  kick(m, n, phi, (0.5 * dt) * s0);
  expansion(m, 0.5 * dt, hubble);
  orc_step_dt(m, step_index, dt / a_mid);
  expansion(m, 0.5 * dt, hubble);
  density_source(m, n, four_pi_G, f);
  orc_mg_solve(n[0], n[1], n[2], h, f, phi, ncycles, nu1, nu2, NULL);
  kick(m, n, phi, (0.5 * dt) * s1);
  free(f);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Test hooks                                                          */
/* ------------------------------------------------------------------ */

void orc_riemann(const double* gas, int iters, const double* WLs, const double* WRs, double* state_out,
                 double* flux_out, double* pstar_out, double* ustar_out) {
  consts_t K = make_consts(gas[0], 0.0, gas[1], iters);
  riemann(&K, WLs, WRs, state_out, flux_out, pstar_out, ustar_out);
}

void orc_pencil_flux(const double* gas, int iters, double nu, int n, const double* U, double* flux_out) {
  consts_t K = make_consts(gas[0], gas[1], gas[2], iters);
  const double* in[5];
  double* out[5];
  for (int v = 0; v < 5; v++) {
    in[v] = U + (int64_t)v * n;
    out[v] = flux_out + (int64_t)v * (n - 5);
  }
  pencil(&K, nu, n, in, out, NULL);
}

/* ------------------------------------------------------------------ */
/* Remesh (Sec. II-B "Refine"; the paper's blast runs refine adaptively) */
/* ------------------------------------------------------------------ */

/* Indicator of one leaf: the largest relative density jump across a cell,
 * max over active cells and axes of |rho(+1) - rho(-1)| / (2 rho).  Reads
 * refreshed ghosts at the block boundary. */
void orc_indicator(const orc_mesh* m, double* out) {
  const int N = m->N, M = m->M;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < m->nleaf; s++) {
    const double* B = block_ptr(m, s);
    double best = 0.0;
    for (int c = G; c < G + N; c++)
      for (int b = G; b < G + N; b++)
        for (int a = G; a < G + N; a++) {
          const double r0 = B[cell(M, 0, a, b, c)];
          const double sx = fabs(B[cell(M, 0, a + 1, b, c)] - B[cell(M, 0, a - 1, b, c)]) / (2.0 * r0);
          const double sy = fabs(B[cell(M, 0, a, b + 1, c)] - B[cell(M, 0, a, b - 1, c)]) / (2.0 * r0);
          const double sz = fabs(B[cell(M, 0, a, b, c + 1)] - B[cell(M, 0, a, b, c - 1)]) / (2.0 * r0);
          best = sx > best ? sx : best;
          best = sy > best ? sy : best;
          best = sz > best ? sz : best;
        }
    out[s] = best;
  }
}

typedef struct { double S; int32_t key[4]; int64_t leaf; } cand_t;

/* Refinement candidates: larger indicator first; ties by (level, z, y, x). */
static int cand_cmp(const void* pa, const void* pb) {
  const cand_t* a = (const cand_t*)pa;
  const cand_t* b = (const cand_t*)pb;
  if (a->S != b->S) return a->S > b->S ? -1 : 1;
  const int order[4] = {0, 3, 2, 1};
  for (int q = 0; q < 4; q++)
    if (a->key[order[q]] != b->key[order[q]]) return a->key[order[q]] < b->key[order[q]] ? -1 : 1;
  return 0;
}

/* Coarsening candidates (parents): finer first; ties by (z, y, x). */
static int par_cmp(const void* pa, const void* pb) {
  const int32_t* a = (const int32_t*)pa;
  const int32_t* b = (const int32_t*)pb;
  if (a[0] != b[0]) return a[0] > b[0] ? -1 : 1;
  for (int q = 3; q >= 1; q--)
    if (a[q] != b[q]) return a[q] < b[q] ? -1 : 1;
  return 0;
}

static int64_t count_leaves(const orc_mesh* m) {
  int64_t n = 0;
  for (int l = 0; l < m->nlev; l++) {
    int64_t cnt = (int64_t)m->ext[l][0] * m->ext[l][1] * m->ext[l][2];
    for (int64_t q = 0; q < cnt; q++) n += m->state[l][q] == LEAF;
  }
  return n;
}

static int balanced(const orc_mesh* m) {
  for (int l = 2; l < m->nlev; l++)
    for (int k = 0; k < m->ext[l][2]; k++)
      for (int j = 0; j < m->ext[l][1]; j++)
        for (int i = 0; i < m->ext[l][0]; i++) {
          if (m->state[l][nidx(m, l, i, j, k)] != LEAF) continue;
          for (int q = 0; q < 27; q++) {
            if (q == 13) continue;
            int p[3] = {i + q % 3 - 1, j + (q / 3) % 3 - 1, k + q / 9 - 1};
            if (!wrap_block(m, l, 0, &p[0]) || !wrap_block(m, l, 1, &p[1]) || !wrap_block(m, l, 2, &p[2]))
              continue;
            if (l - covering_level(m, l, p) >= 2) return 0;
          }
        }
  return 1;
}

static void save_states(const orc_mesh* m, unsigned char** dst) {
  for (int l = 0; l < m->nlev; l++) {
    size_t n = (size_t)m->ext[l][0] * m->ext[l][1] * m->ext[l][2];
    memcpy(dst[l], m->state[l], n);
  }
}
static void load_states(orc_mesh* m, unsigned char** src) {
  for (int l = 0; l < m->nlev; l++) {
    size_t n = (size_t)m->ext[l][0] * m->ext[l][1] * m->ext[l][2];
    memcpy(m->state[l], src[l], n);
  }
}

/* Remesh.  Reading of the refinement rule (the paper names Refine, not its
 * criterion):
 *   1. S_b on refreshed data;
 *   2. every leaf with S_b > refine_slope below the deepest level is a
 *      candidate; in (S_b descending, key) order a candidate is refined
 *      together with the minimal refinement that restores 2:1 balance,
 *      accepted only if every node so refined was a leaf before this remesh
 *      (at most one level of refinement per remesh) and the leaf count stays
 *      <= max_blocks; otherwise it is refused and counted;
 *   3. then, finer first, each octet of leaves that were all leaves before,
 *      all with S_b < coarsen_slope, is merged if 2:1 balance still holds;
 *   4. data: kept leaves copy, new children prolong from their parent (the
 *      refresh prolongation formula, on refreshed parent data), merged
 *      parents restrict their 8 children. */
int orc_remesh(orc_mesh* m, double refine_slope, double coarsen_slope, int64_t max_blocks, orc_mesh** out,
               int64_t* stats) {
  *out = NULL;
  stats[0] = stats[1] = stats[2] = 0;
  orc_refresh(m);
  double* S = (double*)malloc((size_t)m->nleaf * sizeof(double));
  orc_indicator(m, S);
  /* the tree before remesh */
  unsigned char* orig[ORC_MAXLEV];
  unsigned char* keep[ORC_MAXLEV];
  for (int l = 0; l < m->nlev; l++) {
    size_t n = (size_t)m->ext[l][0] * m->ext[l][1] * m->ext[l][2];
    orig[l] = (unsigned char*)malloc(n);
    keep[l] = (unsigned char*)malloc(n);
  }
  save_states(m, orig);
  /* 2. refinement */
  cand_t* cand = (cand_t*)malloc((size_t)m->nleaf * sizeof(cand_t));
  int64_t nc = 0;
  for (int64_t s = 0; s < m->nleaf; s++)
    if (S[s] > refine_slope && m->key[4 * s] < m->d.max_level) {
      cand[nc].S = S[s];
      memcpy(cand[nc].key, m->key + 4 * s, sizeof cand[nc].key);
      cand[nc].leaf = s;
      nc++;
    }
  qsort(cand, (size_t)nc, sizeof(cand_t), cand_cmp);
  for (int64_t q = 0; q < nc; q++) {
    const int32_t* k = cand[q].key;
    if (m->state[k[0]][nidx(m, k[0], k[1], k[2], k[3])] != LEAF) continue; /* refined by an earlier closure */
    save_states(m, keep);
    refine_node(m, k[0], k[1], k[2], k[3]);
    balance(m);
    int ok = count_leaves(m) <= max_blocks;
    for (int l = 0; l < m->nlev && ok; l++) {
      int64_t n = (int64_t)m->ext[l][0] * m->ext[l][1] * m->ext[l][2];
      for (int64_t p = 0; p < n; p++)
        if (m->state[l][p] == REFINED && keep[l][p] != REFINED && orig[l][p] != LEAF) { ok = 0; break; }
    }
    if (!ok) {
      load_states(m, keep);
      stats[2]++;
    }
  }
  for (int l = 0; l < m->nlev; l++) {
    int64_t n = (int64_t)m->ext[l][0] * m->ext[l][1] * m->ext[l][2];
    for (int64_t p = 0; p < n; p++) stats[0] += (m->state[l][p] == REFINED && orig[l][p] != REFINED);
  }
  /* 3. coarsening */
  int64_t npar = 0;
  int32_t* par = (int32_t*)malloc((size_t)(4 * m->nleaf + 4) * sizeof(int32_t));
  for (int l = 0; l + 1 < m->nlev; l++)
    for (int k = 0; k < m->ext[l][2]; k++)
      for (int j = 0; j < m->ext[l][1]; j++)
        for (int i = 0; i < m->ext[l][0]; i++) {
          if (m->state[l][nidx(m, l, i, j, k)] != REFINED) continue;
          int ok = 1;
          for (int c = 0; c < 8 && ok; c++) {
            int ci = 2 * i + (c & 1), cj = 2 * j + ((c >> 1) & 1), ck = 2 * k + (c >> 2);
            int64_t p = nidx(m, l + 1, ci, cj, ck);
            if (m->state[l + 1][p] != LEAF || orig[l + 1][p] != LEAF) ok = 0;
            else if (!(S[m->leaf_at[l + 1][p]] < coarsen_slope)) ok = 0;
          }
          if (ok) {
            par[4 * npar] = l; par[4 * npar + 1] = i; par[4 * npar + 2] = j; par[4 * npar + 3] = k;
            npar++;
          }
        }
  qsort(par, (size_t)npar, 4 * sizeof(int32_t), par_cmp);
  for (int64_t q = 0; q < npar; q++) {
    const int32_t* e = par + 4 * q;
    int l = e[0];
    save_states(m, keep);
    m->state[l][nidx(m, l, e[1], e[2], e[3])] = LEAF;
    for (int c = 0; c < 8; c++)
      m->state[l + 1][nidx(m, l + 1, 2 * e[1] + (c & 1), 2 * e[2] + ((c >> 1) & 1), 2 * e[3] + (c >> 2))] = ABSENT;
    if (balanced(m)) stats[1]++;
    else load_states(m, keep);
  }
  /* 4. new mesh and data migration */
  int64_t nnew = count_leaves(m);
  int32_t* keys = (int32_t*)malloc((size_t)(4 * nnew) * sizeof(int32_t));
  int64_t w = 0;
  for (int l = 0; l < m->nlev; l++)
    for (int k = 0; k < m->ext[l][2]; k++)
      for (int j = 0; j < m->ext[l][1]; j++)
        for (int i = 0; i < m->ext[l][0]; i++)
          if (m->state[l][nidx(m, l, i, j, k)] == LEAF) {
            keys[4 * w] = l; keys[4 * w + 1] = i; keys[4 * w + 2] = j; keys[4 * w + 3] = k;
            w++;
          }
  /* restore the old tree in m (its leaf table still describes its data) */
  load_states(m, orig);
  orc_mesh* nm = NULL;
  int rc = orc_create_from_leaves(&m->d, nnew, keys, &nm);
  if (rc == 0) {
    const int N = m->N, M = m->M;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nm->nleaf; s++) {
      const int32_t* kk = nm->key + 4 * s;
      const int l = kk[0];
      double* D = block_ptr(nm, s);
      if (orig[l][nidx(m, l, kk[1], kk[2], kk[3])] == LEAF) {
        const double* Sb = block_ptr(m, m->leaf_at[l][nidx(m, l, kk[1], kk[2], kk[3])]);
        for (int f = 0; f < m->nf; f++)
          for (int c = G; c < G + N; c++)
            for (int b = G; b < G + N; b++)
              for (int a = G; a < G + N; a++) D[cell(M, f, a, b, c)] = Sb[cell(M, f, a, b, c)];
      } else if (l > 0 && orig[l - 1][nidx(m, l - 1, kk[1] >> 1, kk[2] >> 1, kk[3] >> 1)] == LEAF) {
        /* new child of a refined leaf: prolong from the parent */
        const double* C = block_ptr(m, m->leaf_at[l - 1][nidx(m, l - 1, kk[1] >> 1, kk[2] >> 1, kk[3] >> 1)]);
        const int co[3] = {kk[1] & 1, kk[2] & 1, kk[3] & 1};
        for (int c = 0; c < N; c++)
          for (int b = 0; b < N; b++)
            for (int a = 0; a < N; a++) {
              const int fa[3] = {a, b, c};
              int lc[3];
              double o[3];
              for (int ax = 0; ax < 3; ax++) {
                lc[ax] = (co[ax] * N + fa[ax]) / 2 + G;
                o[ax] = (fa[ax] & 1) ? 1.0 : -1.0;
              }
              for (int f = 0; f < m->nf; f++) {
                double u0 = C[cell(M, f, lc[0], lc[1], lc[2])];
                double sx = minmod(C[cell(M, f, lc[0] + 1, lc[1], lc[2])] - u0, u0 - C[cell(M, f, lc[0] - 1, lc[1], lc[2])]);
                double sy = minmod(C[cell(M, f, lc[0], lc[1] + 1, lc[2])] - u0, u0 - C[cell(M, f, lc[0], lc[1] - 1, lc[2])]);
                double sz = minmod(C[cell(M, f, lc[0], lc[1], lc[2] + 1)] - u0, u0 - C[cell(M, f, lc[0], lc[1], lc[2] - 1)]);
                D[cell(M, f, a + G, b + G, c + G)] =
                    ((u0 + (0.25 * o[0]) * sx) + (0.25 * o[1]) * sy) + (0.25 * o[2]) * sz;
              }
            }
      } else {
        /* merged parent: restrict the 8 old children */
        for (int c = 0; c < N; c++)
          for (int b = 0; b < N; b++)
            for (int a = 0; a < N; a++) {
              const int fa[3] = {a, b, c};
              for (int f = 0; f < m->nf; f++) {
                double v[8];
                for (int q = 0; q < 8; q++) {
                  int64_t gq[3];
                  for (int ax = 0; ax < 3; ax++)
                    gq[ax] = 2 * ((int64_t)kk[1 + ax] * N + fa[ax]) + ((q >> ax) & 1);
                  v[q] = leaf_value(m, l + 1, gq, f);
                }
                D[cell(M, f, a + G, b + G, c + G)] = restrict8(v);
              }
            }
      }
    }
    nm->floors = m->floors;
  }
  for (int l = 0; l < m->nlev; l++) {
    free(orig[l]);
    free(keep[l]);
  }
  free(S); free(cand); free(par); free(keys);
  if (rc != 0) return rc;
  *out = nm;
  return 0;
}
