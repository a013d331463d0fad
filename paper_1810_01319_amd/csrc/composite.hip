// composite.hip -- gfx950 kernels of mg0 on the octree.
//
// The gravity Method's multigrid solver (paper Sec. II-C) on the array of
// octrees (Sec. II-B): the composite-grid Poisson operator on the leaves of
// a refined periodic mesh and the pieces of its V-cycle over the hierarchy
// of coarsened meshes (Omega_l: leaves coarser than l and every octree node
// of level l), each stored like a one-field state (per leaf M^3 padded
// values x, N^3 right-hand side b and operator values L).
//
// Operator: L = (S - 6 x) (1/h^2), S = ((W + E) + (S + N)) + (B + T) from
// ghosts refreshed with linear interpolation over coarser leaves; at a
// coarse cell's face onto finer leaves the coarse difference quotient
// F_c = (g_c - x_c) (1/h) is replaced by the mean of the four fine cells'
// quotients across the face, outward from the coarse cell,
// F_k = (x_k - g_k) (1/h_f):  L += ((((F00 + F10) + (F01 + F11)) 0.25) - F_c)
// (1/h), axes x, y, z in turn.  The fine quotients pass through the plan's
// coarse-fine face slots (first N^2 values of a slot, lower transverse axis
// fastest), as the sweeps' fluxes do for the reflux.
//
// Built with -ffp-contract=off: each formula rounds exactly as written.
#include <hip/hip_runtime.h>

#include "composite.hpp"

namespace amr {

namespace {

constexpr int G = kGhost;
constexpr int kRed = 256;

inline unsigned grid_for(int64_t n, int b) { return unsigned((n + b - 1) / b); }

__device__ __forceinline__ double lvl_dx(const InstParams& ip, int N, int l) {
  return 1.0 / (double)((int64_t)ip.root[0] * N << l);
}

// 7-point part of L on the active cells of colour col (-1: all).
template <int N>
__global__ void __launch_bounds__(256) cz_lap(const double* __restrict__ x, double* __restrict__ Lo, DevPlan P,
                                              int col) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, b = (q / N) % N, c = q / (N * N);
  if (col >= 0 && ((a + b + c) & 1) != col) return;
  const BlockInfo bi = P.blocks[s];
  const double h = lvl_dx(P.inst[bi.inst], N, bi.level);
  const double ih2 = 1.0 / (h * h);
  const double* X = x + int64_t(s) * M3 + (int64_t(c + G) * M + (b + G)) * M + (a + G);
  const double S = ((X[-1] + X[1]) + (X[-M] + X[M])) + (X[-M * M] + X[M * M]);
  Lo[t] = (S - 6.0 * X[0]) * ih2;
}

// Fine side of every coarse-fine face: (x_k - g_k) (1/h_f) of each face cell
// into the face's slot.  One thread per (leaf with a coarser neighbour,
// face, face cell).
template <int N>
__global__ void __launch_bounds__(256) cz_fine_faces(const double* __restrict__ x, DevPlan P) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N2 = N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.np2 * 6 * N2) return;
  const int w = int(t / (6 * N2));
  const int r = int(t - int64_t(w) * 6 * N2);
  const int face = r / N2, cellq = r - face * N2;
  const int dir = face >> 1, side = face & 1;
  const int s = P.p2list[w];
  const int code = 13 + (side ? 1 : -1) * (dir == 0 ? 1 : (dir == 1 ? 3 : 9));
  if (P.nbr[27 * int64_t(s) + code].kind != NBR_COARSE) return;
  const int slot = P.faceslot[6 * int64_t(s) + face];
  const int t1 = cellq % N, t2 = cellq / N;  // along the lower / higher transverse axis
  const int a1 = dir == 0 ? 1 : 0, a2 = dir == 2 ? 1 : 2;
  int p[3];
  p[dir] = side ? N - 1 : 0;
  p[a1] = t1;
  p[a2] = t2;
  const int64_t stride[3] = {1, M, int64_t(M) * M};
  const double* X = x + int64_t(s) * M3 + (int64_t(p[2] + G) * M + (p[1] + G)) * M + (p[0] + G);
  const double g = X[side ? stride[dir] : -stride[dir]];
  const BlockInfo bi = P.blocks[s];
  const double ihf = 1.0 / lvl_dx(P.inst[bi.inst], N, bi.level);
  P.faces[int64_t(slot) * P.nf * N2 + cellq] = (X[0] - g) * ihf;
}

// Coarse side of the coarse-fine faces normal to DIR: L += (Fbar - F_c)
// (1/h) on the face cells of colour col (-1: all).
template <int N, int DIR>
__global__ void __launch_bounds__(256) cz_coarse_faces(const double* __restrict__ x, double* __restrict__ Lo,
                                                       DevPlan P, int col) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N2 = N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nreflux[DIR] * N2) return;
  const int k = int(t / N2);
  const int cellq = int(t - int64_t(k) * N2);
  const RefluxTask T = P.reflux[DIR][k];
  const int t1 = cellq % N, t2 = cellq / N;
  constexpr int A1 = DIR == 0 ? 1 : 0, A2 = DIR == 2 ? 1 : 2;
  int p[3];
  p[DIR] = T.side ? N - 1 : 0;
  p[A1] = t1;
  p[A2] = t2;
  if (col >= 0 && ((p[0] + p[1] + p[2]) & 1) != col) return;
  constexpr int64_t SD = DIR == 0 ? 1 : (DIR == 1 ? M : int64_t(M) * M);
  const double* X = x + int64_t(T.leaf) * M3 + (int64_t(p[2] + G) * M + (p[1] + G)) * M + (p[0] + G);
  const BlockInfo bi = P.blocks[T.leaf];
  const double ih = 1.0 / lvl_dx(P.inst[bi.inst], N, bi.level);
  const double Fc = (X[T.side ? SD : -SD] - X[0]) * ih;
  const int hA = t1 >= N / 2, hB = t2 >= N / 2;
  const double* Q = P.faces + int64_t(T.slot_f[hA + 2 * hB]) * P.nf * N2;
  const int f1 = 2 * t1 - hA * N, f2 = 2 * t2 - hB * N;
  const double Fbar = ((Q[f2 * N + f1] + Q[f2 * N + f1 + 1]) + (Q[(f2 + 1) * N + f1] + Q[(f2 + 1) * N + f1 + 1])) * 0.25;
  const int64_t o = int64_t(T.leaf) * N * N2 + (int64_t(p[2]) * N + p[1]) * N + p[0];
  Lo[o] = Lo[o] + (Fbar - Fc) * ih;
}

// Red-black update of colour col: x -= (b - L) / D, D = (6 + n_cf) (1/h^2).
template <int N>
__global__ void __launch_bounds__(256) cz_update(double* __restrict__ x, const double* __restrict__ b,
                                                 const double* __restrict__ Lo, DevPlan P, int col) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, bb = (q / N) % N, c = q / (N * N);
  if (((a + bb + c) & 1) != col) return;
  const BlockInfo bi = P.blocks[s];
  const double h = lvl_dx(P.inst[bi.inst], N, bi.level);
  const double ih2 = 1.0 / (h * h);
  const int loc[3] = {a, bb, c};
  int ncf = 0;
  for (int d = 0; d < 3; d++) {
    if (loc[d] == 0 && (bi.rflx >> (2 * d)) & 1) ncf++;
    if (loc[d] == N - 1 && (bi.rflx >> (2 * d + 1)) & 1) ncf++;
  }
  const double r = b[t] - Lo[t];
  const double D = (double)(6 + ncf) * ih2;
  double* X = x + int64_t(s) * M3 + (int64_t(c + G) * M + (bb + G)) * M + (a + G);
  *X = *X - r / D;
}

// L <- b - L (the residual) on every active cell.
__global__ void __launch_bounds__(256) cz_resid(const double* __restrict__ b, double* __restrict__ Lo, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) Lo[t] = b[t] - Lo[t];
}

// Restriction of the finer stage's residual Lf into the coarser stage's
// right-hand side bc: per coarse-stage leaf a copy or the mean of its 8
// children (summed x fastest, then y, then z, in pairs).
template <int N>
__global__ void __launch_bounds__(256) cz_restrict(const double* __restrict__ Lf, double* __restrict__ bc,
                                                   const MigrTask* __restrict__ tasks, int64_t nleaf) {
  constexpr int N3 = N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, b = (q / N) % N, c = q / (N * N);
  const MigrTask T = tasks[s];
  if (T.kind == MIGR_COPY) {
    bc[t] = Lf[int64_t(T.src[0]) * N3 + q];
    return;
  }
  const int fx = 2 * a, fy = 2 * b, fz = 2 * c;
  const int ch = (fx / N) + 2 * (fy / N) + 4 * (fz / N);
  const int la = fx % N, lb = fy % N, lc = fz % N;
  const double* Q = Lf + int64_t(T.src[ch]) * N3 + (int64_t(lc) * N + lb) * N + la;
  const double v0 = Q[0], v1 = Q[1], v2 = Q[N], v3 = Q[N + 1];
  const double v4 = Q[N * N], v5 = Q[N * N + 1], v6 = Q[N * N + N], v7 = Q[N * N + N + 1];
  bc[t] = (((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7))) * 0.125;
}

// x of the finer stage += the coarser stage's correction e (ghosts
// refreshed): a copy, or from the parent cell with central slopes.
template <int N>
__global__ void __launch_bounds__(256) cz_prolong_add(const double* __restrict__ e, double* __restrict__ x,
                                                      const MigrTask* __restrict__ tasks, int64_t nleaf) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, b = (q / N) % N, c = q / (N * N);
  const MigrTask T = tasks[s];
  double v;
  if (T.kind == MIGR_COPY) {
    v = e[int64_t(T.src[0]) * M3 + (int64_t(c + G) * M + (b + G)) * M + (a + G)];
  } else {
    const int gx = (T.co & 1) * N + a, gy = ((T.co >> 1) & 1) * N + b, gz = (T.co >> 2) * N + c;
    const double* E = e + int64_t(T.src[0]) * M3 + (int64_t(gz / 2 + G) * M + (gy / 2 + G)) * M + (gx / 2 + G);
    const double ox = (gx & 1) ? 0.25 : -0.25;
    const double oy = (gy & 1) ? 0.25 : -0.25;
    const double oz = (gz & 1) ? 0.25 : -0.25;
    const double u0 = E[0];
    const double sx = 0.5 * (E[1] - E[-1]);
    const double sy = 0.5 * (E[M] - E[-M]);
    const double sz = 0.5 * (E[M * M] - E[-M * M]);
    v = ((u0 + ox * sx) + oy * sy) + oz * sz;
  }
  double* X = x + int64_t(s) * M3 + (int64_t(c + G) * M + (b + G)) * M + (a + G);
  *X = *X + v;
}

// Active cells between block layout (N^3 per leaf) and the padded layout.
template <int N, bool IN>
__global__ void __launch_bounds__(256) cz_copy(const double* __restrict__ src, double* __restrict__ dst,
                                               int64_t nleaf, const double* __restrict__ sub) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, b = (q / N) % N, c = q / (N * N);
  const int64_t p = int64_t(s) * M3 + (int64_t(c + G) * M + (b + G)) * M + (a + G);
  if (IN) dst[p] = src[t];
  else dst[t] = sub ? src[p] - *sub : src[p];
}

__global__ void __launch_bounds__(256) cz_fill(double* __restrict__ a, int64_t n, double v) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) a[t] = v;
}

__device__ __forceinline__ double group_sum(double v) {
  __shared__ double red[kRed];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kRed / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// parts[s] = 8^-level(s) * (sum over leaf s of v (SQ: v^2)); v in block
// layout (PAD false) or the active cells of the padded layout.  One
// workgroup per leaf; fixed summation order.
template <int N, bool SQ, bool PAD>
__global__ void __launch_bounds__(kRed) cz_leaf_sums(const double* __restrict__ v, DevPlan P,
                                                     double* __restrict__ parts) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int q = threadIdx.x; q < N3; q += kRed) {
    const int a = q % N, b = (q / N) % N, c = q / (N * N);
    const double y = PAD ? v[int64_t(s) * M3 + (int64_t(c + G) * M + (b + G)) * M + (a + G)] : v[int64_t(s) * N3 + q];
    acc = acc + (SQ ? y * y : y);
  }
  const double tot = group_sum(acc);
  if (threadIdx.x == 0) parts[s] = ldexp(1.0, -3 * P.blocks[s].level) * tot;
}

// out[0] = scale * sum of parts[0..n) (SQRT: its square root), fixed order.
template <bool SQRT>
__global__ void __launch_bounds__(kRed) cz_sum_final(const double* __restrict__ parts, int64_t n, double scale,
                                                     double* __restrict__ out) {
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kRed) acc = acc + parts[i];
  const double tot = group_sum(acc);
  if (threadIdx.x == 0) out[0] = SQRT ? sqrt(scale * tot) : scale * tot;
}

__global__ void __launch_bounds__(256) cz_sub(double* __restrict__ a, int64_t n, const double* __restrict__ m) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) a[t] = a[t] - *m;
}

template <int N>
__global__ void __launch_bounds__(256) cz_density(const double* __restrict__ U, double* __restrict__ b, DevPlan P,
                                                  double fpg) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, bb = (q / N) % N, c = q / (N * N);
  b[t] = fpg * U[int64_t(s) * P.nf * M3 + (int64_t(c + G) * M + (bb + G)) * M + (a + G)];
}

// Half kick with g = -grad(x), central differences at the cell's level
// (x's ghosts refreshed): momentum + hdt rho g, energy + (ke' - ke),
// hdt = (dt/2) scale; the arithmetic of the uniform mesh's kick.
template <int N>
__global__ void __launch_bounds__(256) cz_kick(double* __restrict__ U, const double* __restrict__ x, DevPlan P,
                                               const double* __restrict__ dtv, double scale) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, b = (q / N) % N, c = q / (N * N);
  const BlockInfo bi = P.blocks[s];
  const double inv2h = 1.0 / (2.0 * lvl_dx(P.inst[bi.inst], N, bi.level));
  const int64_t o = (int64_t(c + G) * M + (b + G)) * M + (a + G);
  const double* X = x + int64_t(s) * M3 + o;
  double gv[3];
  gv[0] = (X[-1] - X[1]) * inv2h;
  gv[1] = (X[-M] - X[M]) * inv2h;
  gv[2] = (X[-M * M] - X[M * M]) * inv2h;
  double* B = U + int64_t(s) * P.nf * M3 + o;
  const double hdt = (0.5 * dtv[0]) * scale;
  const double rho = B[0];
  double mo[3] = {B[M3], B[2 * M3], B[3 * M3]};
  double E = B[4 * M3];
  const double ir = 1.0 / rho;
  double u[3], u2[3];
#pragma unroll
  for (int ax = 0; ax < 3; ax++) u[ax] = mo[ax] * ir;
  const double ke = (0.5 * rho) * ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
#pragma unroll
  for (int ax = 0; ax < 3; ax++) {
    mo[ax] = mo[ax] + hdt * (rho * gv[ax]);
    u2[ax] = mo[ax] * ir;
  }
  const double ke2 = (0.5 * rho) * ((u2[0] * u2[0] + u2[1] * u2[1]) + u2[2] * u2[2]);
  E = E + (ke2 - ke);
#pragma unroll
  for (int ax = 0; ax < 3; ax++) B[(1 + ax) * M3] = mo[ax];
  B[4 * M3] = E;
}

template <int N>
hipError_t ops_n(const CzOp& op, hipStream_t st) {
  constexpr int N3 = N * N * N;
  const DevPlan& P = op.P;
  const int64_t n = P.nleaf * int64_t(N3);
  const dim3 b(256);
  switch (op.kind) {
    case CZ_OPERATOR: {
      if (P.np2 > 0)
        hipLaunchKernelGGL((cz_fine_faces<N>), dim3(grid_for(P.np2 * 6 * N * N, 256)), b, 0, st, op.x, P);
      hipLaunchKernelGGL((cz_lap<N>), dim3(grid_for(n, 256)), b, 0, st, op.x, op.L, P, op.col);
      if (P.nreflux[0] > 0)
        hipLaunchKernelGGL((cz_coarse_faces<N, 0>), dim3(grid_for(P.nreflux[0] * N * N, 256)), b, 0, st, op.x, op.L, P, op.col);
      if (P.nreflux[1] > 0)
        hipLaunchKernelGGL((cz_coarse_faces<N, 1>), dim3(grid_for(P.nreflux[1] * N * N, 256)), b, 0, st, op.x, op.L, P, op.col);
      if (P.nreflux[2] > 0)
        hipLaunchKernelGGL((cz_coarse_faces<N, 2>), dim3(grid_for(P.nreflux[2] * N * N, 256)), b, 0, st, op.x, op.L, P, op.col);
      break;
    }
    case CZ_UPDATE:
      hipLaunchKernelGGL((cz_update<N>), dim3(grid_for(n, 256)), b, 0, st, op.x, op.b, op.L, P, op.col);
      break;
    case CZ_RESID:
      hipLaunchKernelGGL(cz_resid, dim3(grid_for(n, 256)), b, 0, st, op.b, op.L, n);
      break;
    case CZ_RESTRICT:  // P: the coarser stage
      hipLaunchKernelGGL((cz_restrict<N>), dim3(grid_for(n, 256)), b, 0, st, op.L, op.b, op.tasks, P.nleaf);
      break;
    case CZ_PROLONG:  // P: the finer stage
      hipLaunchKernelGGL((cz_prolong_add<N>), dim3(grid_for(n, 256)), b, 0, st, op.e, op.x, op.tasks, P.nleaf);
      break;
    case CZ_COPY_IN:
      hipLaunchKernelGGL((cz_copy<N, true>), dim3(grid_for(n, 256)), b, 0, st, op.src, op.x, P.nleaf, nullptr);
      break;
    case CZ_COPY_OUT:
      hipLaunchKernelGGL((cz_copy<N, false>), dim3(grid_for(n, 256)), b, 0, st, op.x, op.dst, P.nleaf, op.scal);
      break;
    case CZ_ZERO: {
      constexpr int M = N + 2 * G;
      const int64_t np = P.nleaf * int64_t(M) * M * M;
      hipLaunchKernelGGL(cz_fill, dim3(grid_for(np, 256)), b, 0, st, op.x, np, 0.0);
      break;
    }
    case CZ_MEAN_SUB:  // b -= its volume-weighted mean
      hipLaunchKernelGGL((cz_leaf_sums<N, false, false>), dim3(unsigned(P.nleaf)), dim3(kRed), 0, st, op.b, P, op.parts);
      hipLaunchKernelGGL(cz_sum_final<false>, dim3(1), dim3(kRed), 0, st, op.parts, P.nleaf, op.scale, op.scal);
      hipLaunchKernelGGL(cz_sub, dim3(grid_for(n, 256)), b, 0, st, op.b, n, op.scal);
      break;
    case CZ_MEAN_PADDED:  // scal = volume-weighted mean of x's active cells
      hipLaunchKernelGGL((cz_leaf_sums<N, false, true>), dim3(unsigned(P.nleaf)), dim3(kRed), 0, st, op.x, P, op.parts);
      hipLaunchKernelGGL(cz_sum_final<false>, dim3(1), dim3(kRed), 0, st, op.parts, P.nleaf, op.scale, op.scal);
      break;
    case CZ_DENSITY:
      hipLaunchKernelGGL((cz_density<N>), dim3(grid_for(n, 256)), b, 0, st, op.U, op.b, P, op.fpg);
      break;
    case CZ_KICK:
      hipLaunchKernelGGL((cz_kick<N>), dim3(grid_for(n, 256)), b, 0, st, op.U, op.x, P, op.dt, op.scale);
      break;
    case CZ_NORM:  // scal = sqrt(volume-weighted sum of L^2)
      hipLaunchKernelGGL((cz_leaf_sums<N, true, false>), dim3(unsigned(P.nleaf)), dim3(kRed), 0, st, op.L, P, op.parts);
      hipLaunchKernelGGL(cz_sum_final<true>, dim3(1), dim3(kRed), 0, st, op.parts, P.nleaf, 1.0, op.scal);
      break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t cz_launch(const CzOp& op, hipStream_t st) {
  switch (op.P.N) {
    case 8: return ops_n<8>(op, st);
    case 16: return ops_n<16>(op, st);
    case 32: return ops_n<32>(op, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace amr
