// poisson.hip -- gfx950 kernels of the mg0 Poisson solver.
//
// The gravity Method's geometric multigrid V-cycle (paper Sec. II-C; the
// self-gravity solver of its uniform-mesh cosmology test, Sec. III): the
// 7-point Laplacian of phi equals f on a uniform periodic mesh.  Each level
// is one global grid stored split by colour: cell (i, j, k) of colour
// c = (i + j + k) mod 2 sits at c n/2 + (k ny + j) nx/2 + i/2, so a colour
// pass reads the other colour and writes its own with unit stride across
// lanes and moves no line of the colour it skips.  Level l+1 halves every axis of level l
// and exists while all of level l's axes are multiples of 4.  Red-black
// Gauss-Seidel smoothing (red = (i + j + k) even first), residual restriction
// by the mean of the 8 children, trilinear prolongation of the correction,
// 64 red-black sweeps on the coarsest level in one workgroup's LDS.  Every
// cell update is a fixed expression, so the smoothing, transfer and coarse
// kernels give the same bits in any launch shape; the means and residual
// norms are two-stage reductions in a fixed order.
//
// Built with -ffp-contract=off: each formula rounds exactly as written.
#include <hip/hip_runtime.h>

#include <mutex>

#include "poisson.hpp"

#include "expansion_cell.hpp"

namespace amr {

namespace {

constexpr int kRedBlock = 256;     // threads of a reduction workgroup
constexpr int kRedParts = 1024;    // workgroups of the first reduction stage
constexpr int kCoarseThreads = 1024;

struct Lvl {
  double* phi;
  double* f;
  int nx, ny, nz;
  double h;
};

__device__ __forceinline__ int wrap_dn(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wrap_up(int i, int n) { return i == n - 1 ? 0 : i + 1; }

// Storage index of cell (i, j, k) (colour-split layout).
__device__ __forceinline__ int64_t lidx(const Lvl& L, int i, int j, int k) {
  const int64_t half = (int64_t(L.nx) * L.ny * L.nz) >> 1;
  return ((i + j + k) & 1) * half + (int64_t(k) * L.ny + j) * (L.nx >> 1) + (i >> 1);
}

// Cell of storage index t: colour t / (n/2), then z, y, x/2.
__device__ __forceinline__ void lcell(const Lvl& L, int64_t t, int& i, int& j, int& k) {
  const int64_t half = (int64_t(L.nx) * L.ny * L.nz) >> 1;
  const int c = t >= half ? 1 : 0;
  const int64_t r = t - c * half;
  const int hx = L.nx >> 1;
  const int m = int(r % hx);
  const int64_t q = r / hx;
  j = int(q % L.ny);
  k = int(q / L.ny);
  i = 2 * m + ((j + k + c) & 1);
}

// ((W + E) + (S + N)) + (B + T) of phi around (i, j, k), periodic.
__device__ __forceinline__ double nbr_sum(const Lvl& L, const double* p, int i, int j, int k) {
  const double w = p[lidx(L, wrap_dn(i, L.nx), j, k)], e = p[lidx(L, wrap_up(i, L.nx), j, k)];
  const double s = p[lidx(L, i, wrap_dn(j, L.ny), k)], n = p[lidx(L, i, wrap_up(j, L.ny), k)];
  const double b = p[lidx(L, i, j, wrap_dn(k, L.nz))], t = p[lidx(L, i, j, wrap_up(k, L.nz))];
  return ((w + e) + (s + n)) + (b + t);
}

// Workgroup -> (x chunk bx of gx, row j, plane k) over a (gx, ny, nz) grid.
// Workgroups are dealt to the 8 XCDs in turn (linear id mod 8, x fastest),
// each XCD with its own L2.  When ny is a multiple of 8, XCD x takes the band
// of rows j in [x ny/8, (x+1) ny/8), plane after plane: the rows j +- 1 and
// planes k +- 1 that a workgroup reads were then fetched into that XCD's L2
// by its neighbours in the band (with the natural order, row j went to XCD
// j mod 8 and its y neighbours to two other XCDs).
__device__ __forceinline__ void block_row(int gx, int ny, int& bx, int& j, int& k) {
  const unsigned b = blockIdx.x + unsigned(gx) * (blockIdx.y + unsigned(ny) * blockIdx.z);
  if ((ny & 7) == 0) {
    const unsigned x = b & 7u, q = b >> 3, band = unsigned(ny) >> 3;
    bx = int(q % unsigned(gx));
    const unsigned r = q / unsigned(gx);
    j = int(x * band + r % band);
    k = int(r / band);
  } else {
    bx = int(blockIdx.x);
    j = int(blockIdx.y);
    k = int(blockIdx.z);
  }
}

// One colour of a red-black sweep: thread m of row (j, k) updates the
// colour's cell i = 2m + parity.
__global__ void __launch_bounds__(256) mg_rbgs(Lvl L, int color, int gx) {
  const int hx = L.nx >> 1;
  int bx, j, k;
  block_row(gx, L.ny, bx, j, k);
  const int m = int(bx * blockDim.x + threadIdx.x);
  if (m >= hx) return;
  const int i = 2 * m + ((j + k + color) & 1);
  const int64_t half = (int64_t(L.nx) * L.ny * L.nz) >> 1;
  const int64_t c = color * half + (int64_t(k) * L.ny + j) * hx + m;
  const double h2 = L.h * L.h, sixth = 1.0 / 6.0;
  L.phi[c] = (nbr_sum(L, L.phi, i, j, k) - h2 * L.f[c]) * sixth;
}

__device__ __forceinline__ double residual_at(const Lvl& L, int i, int j, int k) {
  const int64_t c = lidx(L, i, j, k);
  const double ih2 = 1.0 / (L.h * L.h);
  return L.f[c] - (nbr_sum(L, L.phi, i, j, k) - 6.0 * L.phi[c]) * ih2;
}

// Coarse right-hand side = mean of the 8 children's residuals (x fastest,
// then y, then z, in pairs); the coarse correction starts from 0.
// Threads run over coarse cells in natural order (x fastest), so that the
// children's reads are contiguous across lanes in the fine colour arrays.
__global__ void __launch_bounds__(256) mg_restrict(Lvl F, Lvl C, int gx) {
  int bx, j, k;
  block_row(gx, C.ny, bx, j, k);  // rows of the coarse level
  const int i = int(bx * blockDim.x + threadIdx.x);
  if (i >= C.nx) return;
  double r[8];
#pragma unroll
  for (int o = 0; o < 8; o++) r[o] = residual_at(F, 2 * i + (o & 1), 2 * j + ((o >> 1) & 1), 2 * k + (o >> 2));
  const int64_t c = lidx(C, i, j, k);
  C.f[c] = (((r[0] + r[1]) + (r[2] + r[3])) + ((r[4] + r[5]) + (r[6] + r[7]))) * 0.125;
  C.phi[c] = 0.0;
}

// Trilinear prolongation of the coarse correction, added to the fine phi:
// one thread per coarse cell (natural order) reads its 27 coarse neighbours
// once and updates its 8 children.
__global__ void __launch_bounds__(256) mg_prolong_add(Lvl C, Lvl F, int gx) {
  int bx, J, K;
  block_row(gx, C.ny, bx, J, K);  // rows of the coarse level
  const int I = int(bx * blockDim.x + threadIdx.x);
  if (I >= C.nx) return;
  const int xs[3] = {wrap_dn(I, C.nx), I, wrap_up(I, C.nx)};
  const int ys[3] = {wrap_dn(J, C.ny), J, wrap_up(J, C.ny)};
  const int zs[3] = {wrap_dn(K, C.nz), K, wrap_up(K, C.nz)};
  double cv[3][3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
      for (int d = 0; d < 3; d++) cv[a][b][d] = C.phi[lidx(C, xs[d], ys[b], zs[a])];
  const double w64 = 1.0 / 64.0;
#pragma unroll
  for (int o = 0; o < 8; o++) {
    const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
    const int sx = ox ? 2 : 0, sy = oy ? 2 : 0, sz = oz ? 2 : 0;  // neighbour towards the child's corner
    const double c0 = cv[1][1][1];
    const double cx = cv[1][1][sx], cy = cv[1][sy][1], cz = cv[sz][1][1];
    const double cxy = cv[1][sy][sx], cxz = cv[sz][1][sx], cyz = cv[sz][sy][1];
    const double cxyz = cv[sz][sy][sx];
    const double v = ((27.0 * c0 + 9.0 * ((cx + cy) + cz)) + (3.0 * ((cxy + cxz) + cyz) + cxyz)) * w64;
    const int64_t fidx = lidx(F, 2 * I + ox, 2 * J + oy, 2 * K + oz);
    F.phi[fidx] = F.phi[fidx] + v;
  }
}

// Coarsest level: 64 red-black sweeps in one workgroup's LDS (at most
// kMgCoarseMax cells), from its phi (0 below the finest level, which is set
// by the restriction; the iterate itself on a one-level grid).
__global__ void __launch_bounds__(kCoarseThreads) mg_coarse_solve(Lvl L) {
  __shared__ double ph[kMgCoarseMax];
  __shared__ double rhs[kMgCoarseMax];
  const int n = L.nx * L.ny * L.nz;  // LDS in natural order (x fastest)
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int i = c % L.nx, j = (c / L.nx) % L.ny, k = c / (L.nx * L.ny);
    ph[c] = L.phi[lidx(L, i, j, k)];
    rhs[c] = L.f[lidx(L, i, j, k)];
  }
  __syncthreads();
  const double h2 = L.h * L.h, sixth = 1.0 / 6.0;
  for (int sweep = 0; sweep < kMgCoarseSweeps; sweep++)
    for (int color = 0; color < 2; color++) {
      for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const int i = c % L.nx, j = (c / L.nx) % L.ny, k = c / (L.nx * L.ny);
        if (((i + j + k) & 1) != color) continue;
        const int row = L.nx, pln = L.nx * L.ny;
        const double w = ph[c - i + wrap_dn(i, L.nx)], e = ph[c - i + wrap_up(i, L.nx)];
        const double s = ph[c + (wrap_dn(j, L.ny) - j) * row], nn = ph[c + (wrap_up(j, L.ny) - j) * row];
        const double b = ph[c + (wrap_dn(k, L.nz) - k) * pln], t = ph[c + (wrap_up(k, L.nz) - k) * pln];
        ph[c] = ((((w + e) + (s + nn)) + (b + t)) - h2 * rhs[c]) * sixth;
      }
      __syncthreads();
    }
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int i = c % L.nx, j = (c / L.nx) % L.ny, k = c / (L.nx * L.ny);
    L.phi[lidx(L, i, j, k)] = ph[c];
  }
}

// Level 0 from the block layout (per leaf N^3 active cells, x fastest): phi
// from pb; f from fb (SRC 0), from fpg times the density of the state U
// (SRC 1: padded blocks of P.nf fields), or left alone (SRC 2).
template <int N, int SRC>
__global__ void __launch_bounds__(256) mg_gather(const double* __restrict__ fb, const double* __restrict__ U,
                                                 double fpg, const double* __restrict__ pb, Lvl L, DevPlan P) {
  constexpr int N3 = N * N * N;
  constexpr int M = N + 2 * kGhost;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, b = (q / N) % N, c = q / (N * N);
  const BlockInfo bi = P.blocks[s];
  const int64_t g = lidx(L, bi.i * N + a, bi.j * N + b, bi.k * N + c);
  if (SRC == 0 || SRC == 3) L.f[g] = fb[t];
  if (SRC == 1)
    L.f[g] = fpg * U[int64_t(s) * P.nf * M * M * M + (int64_t(c + kGhost) * M + (b + kGhost)) * M + (a + kGhost)];
  L.phi[g] = SRC == 3 ? 0.0 : pb[t];
}

// Level 0's phi into the active cells of a padded one-field block layout
// (per leaf M^3), as it is.
template <int N>
__global__ void __launch_bounds__(256) mg_scatter_padded(Lvl L, DevPlan P, double* __restrict__ x) {
  constexpr int N3 = N * N * N;
  constexpr int M = N + 2 * kGhost;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, b = (q / N) % N, c = q / (N * N);
  const BlockInfo bi = P.blocks[s];
  x[int64_t(s) * M * M * M + (int64_t(c + kGhost) * M + (b + kGhost)) * M + (a + kGhost)] =
      L.phi[lidx(L, bi.i * N + a, bi.j * N + b, bi.k * N + c)];
}

// Half kick of the active cells with g = -grad(phi) (central differences of
// level 0's phi, which holds a mean-free potential): momentum + hdt rho g,
// energy + (ke' - ke), hdt = (dt/2) scale (scale 1/a^2 in comoving steps).
// EXP 1: the expansion sources over dt/2 follow the kick in the same pass
// (c = (halfdt/2) H, halfdt = dt/2 on the device); EXP 2: they precede it.
// Each cell's arithmetic is that of the separate kick and expansion kernels.
template <int N, int EXP>
__global__ void __launch_bounds__(256) mg_kick(double* __restrict__ U, Lvl L, DevPlan P,
                                               const double* __restrict__ dtv, double scale,
                                               const double* __restrict__ halfdt, double hubble) {
  constexpr int N3 = N * N * N;
  constexpr int M = N + 2 * kGhost;
  constexpr int64_t M3 = int64_t(M) * M * M;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, b = (q / N) % N, c = q / (N * N);
  const BlockInfo bi = P.blocks[s];
  const int p[3] = {bi.i * N + a, bi.j * N + b, bi.k * N + c};
  const int n[3] = {L.nx, L.ny, L.nz};
  const double inv2h = 1.0 / (2.0 * L.h);
  double gv[3];
#pragma unroll
  for (int ax = 0; ax < 3; ax++) {
    int lo[3] = {p[0], p[1], p[2]}, hi[3] = {p[0], p[1], p[2]};
    lo[ax] = wrap_dn(p[ax], n[ax]);
    hi[ax] = wrap_up(p[ax], n[ax]);
    gv[ax] = (L.phi[lidx(L, lo[0], lo[1], lo[2])] - L.phi[lidx(L, hi[0], hi[1], hi[2])]) * inv2h;
  }
  double* B = U + int64_t(s) * P.nf * M3 + (int64_t(c + kGhost) * M + (b + kGhost)) * M + (a + kGhost);
  const double hdt = (0.5 * dtv[0]) * scale;
  const bool de = P.nf == kFieldsDE;
  const double rho = B[0];
  double mo[3] = {B[M3], B[2 * M3], B[3 * M3]};
  double E = B[4 * M3];
  double ge = EXP != 0 && de ? B[5 * M3] : 0.0;
  unsigned nfl = 0;
  InstParams ip;
  double cexp = 0.0;
  if (EXP != 0) {
    ip = P.inst[bi.inst];
    cexp = (0.5 * halfdt[0]) * hubble;
  }
  if (EXP == 2) nfl += expansion_cell(ip, cexp, de, rho, mo[0], mo[1], mo[2], E, ge);
  {
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
  }
  if (EXP == 1) nfl += expansion_cell(ip, cexp, de, rho, mo[0], mo[1], mo[2], E, ge);
#pragma unroll
  for (int ax = 0; ax < 3; ax++) B[(1 + ax) * M3] = mo[ax];
  B[4 * M3] = E;
  if (EXP != 0 && de) B[5 * M3] = ge;
  if (nfl) atomicAdd(P.counters, (unsigned long long)nfl);
}

// Block layout from level 0, minus the mean held at *mean; level 0 keeps the
// same mean-free values, so a kick right after the solve needs no gather.
template <int N>
__global__ void __launch_bounds__(256) mg_scatter(Lvl L, DevPlan P, const double* __restrict__ mean,
                                                  double* __restrict__ pb) {
  constexpr int N3 = N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const BlockInfo bi = P.blocks[s];
  const int64_t g = lidx(L, bi.i * N + q % N, bi.j * N + (q / N) % N, bi.k * N + q / (N * N));
  const double v = L.phi[g] - *mean;
  pb[t] = v;
  L.phi[g] = v;
}

// dst[0] = factor src[0] (one lane).
__global__ void mg_scale_scalar(const double* __restrict__ src, double* __restrict__ dst, double factor) {
  if (blockIdx.x == 0 && threadIdx.x == 0) dst[0] = factor * src[0];
}

__global__ void __launch_bounds__(256) mg_sub_mean(double* __restrict__ a, int64_t n, const double* __restrict__ mean) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) a[t] = a[t] - *mean;
}

// Workgroup sum in a fixed tree order.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kRedBlock];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// First stage: part b sums the elements b, b + kRedParts kRedBlock, ... of
// each of its lanes' strided sequences (MODE 0: a; MODE 1: the squared
// residual of level L).
template <int MODE>
__global__ void __launch_bounds__(kRedBlock) mg_sum_parts(const double* __restrict__ a, Lvl L, int64_t n,
                                                          double* __restrict__ parts) {
  double s = 0.0;
  for (int64_t t = int64_t(blockIdx.x) * kRedBlock + threadIdx.x; t < n; t += int64_t(kRedParts) * kRedBlock) {
    if (MODE == 0) {
      s += a[t];
    } else {
      int i, j, k;
      lcell(L, t, i, j, k);
      const double r = residual_at(L, i, j, k);
      s += r * r;
    }
  }
  const double b = block_sum(s);
  if (threadIdx.x == 0) parts[blockIdx.x] = b;
}

// Second stage: *out = sum of the parts times scale (MODE 0), or its square
// root (MODE 1).
template <int MODE>
__global__ void __launch_bounds__(kRedBlock) mg_sum_final(const double* __restrict__ parts, double scale,
                                                          double* __restrict__ out) {
  double s = 0.0;
  for (int b = threadIdx.x; b < kRedParts; b += kRedBlock) s += parts[b];
  const double tot = block_sum(s);
  if (threadIdx.x == 0) *out = MODE == 0 ? tot * scale : sqrt(tot);
}

inline unsigned grid_for(int64_t n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

int mg_levels(int nx, int ny, int nz, int sizes[][3]) {
  int n[3] = {nx, ny, nz}, nl = 0;
  while (true) {
    for (int a = 0; a < 3; a++) sizes[nl][a] = n[a];
    nl++;
    if (nl >= kMgMaxLevels || n[0] % 4 || n[1] % 4 || n[2] % 4) break;
    for (int a = 0; a < 3; a++) n[a] /= 2;
  }
  return nl;
}

// The solver's workspace for callers that cannot allocate device memory
// (amr_poisson_solve_static).  Host code never names it: its name on the host
// is a stand-in, not a device address; mg_static_scratch returns the address
// of the current device's copy.
static __device__ __align__(256) unsigned char scratch[kMgStaticScratchBytes];

hipError_t mg_static_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

int64_t mg_workspace_bytes(int nx, int ny, int nz) {
  int sz[kMgMaxLevels][3];
  const int nl = mg_levels(nx, ny, nz, sz);
  int64_t o = 0;
  for (int l = 0; l < nl; l++) o += 2 * ((int64_t(sz[l][0]) * sz[l][1] * sz[l][2] * 8 + 255) / 256 * 256);
  return o + (kRedParts + 64) * 8;
}

namespace {

void levels_in(void* work, int nx, int ny, int nz, double h, Lvl* Ls, int& nl, double*& parts) {
  int sz[kMgMaxLevels][3];
  nl = mg_levels(nx, ny, nz, sz);
  unsigned char* w = static_cast<unsigned char*>(work);
  double hl = h;
  for (int l = 0; l < nl; l++) {
    const int64_t bytes = (int64_t(sz[l][0]) * sz[l][1] * sz[l][2] * 8 + 255) / 256 * 256;
    Ls[l] = Lvl{reinterpret_cast<double*>(w), reinterpret_cast<double*>(w + bytes), sz[l][0], sz[l][1], sz[l][2], hl};
    w += 2 * bytes;
    hl = 2.0 * hl;
  }
  parts = reinterpret_cast<double*>(w);
}

template <int SRC>
void gather_n(const DevPlan& P, const double* fb, const double* U, double fpg, const double* pb, const Lvl& L0,
              hipStream_t st) {
  const int64_t nb = P.nleaf * int64_t(P.N) * P.N * P.N;
  const dim3 g(grid_for(nb, 256)), b(256);
  if (P.N == 8) hipLaunchKernelGGL((mg_gather<8, SRC>), g, b, 0, st, fb, U, fpg, pb, L0, P);
  else if (P.N == 16) hipLaunchKernelGGL((mg_gather<16, SRC>), g, b, 0, st, fb, U, fpg, pb, L0, P);
  else hipLaunchKernelGGL((mg_gather<32, SRC>), g, b, 0, st, fb, U, fpg, pb, L0, P);
}

}  // namespace

namespace {
template <int N>
void kick_n(int exp, dim3 g, dim3 b, hipStream_t st, double* U, const Lvl& L0, const DevPlan& P, const double* dt,
            double scale, const double* halfdt, double hubble) {
  if (exp == 1) hipLaunchKernelGGL((mg_kick<N, 1>), g, b, 0, st, U, L0, P, dt, scale, halfdt, hubble);
  else if (exp == 2) hipLaunchKernelGGL((mg_kick<N, 2>), g, b, 0, st, U, L0, P, dt, scale, halfdt, hubble);
  else hipLaunchKernelGGL((mg_kick<N, 0>), g, b, 0, st, U, L0, P, dt, scale, halfdt, hubble);
}
}  // namespace

hipError_t mg_kick(const DevPlan& P, int nx, int ny, int nz, double h, double* U, const double* phi_blocks,
                   const double* dt, double scale, void* work, hipStream_t st, int exp, const double* halfdt,
                   double hubble, bool level0_current) {
  Lvl Ls[kMgMaxLevels];
  int nl;
  double* parts;
  levels_in(work, nx, ny, nz, h, Ls, nl, parts);
  if (!level0_current) gather_n<2>(P, nullptr, nullptr, 0.0, phi_blocks, Ls[0], st);
  const int64_t nb = P.nleaf * int64_t(P.N) * P.N * P.N;
  const dim3 g(grid_for(nb, 256)), b(256);
  if (P.N == 8) kick_n<8>(exp, g, b, st, U, Ls[0], P, dt, scale, halfdt, hubble);
  else if (P.N == 16) kick_n<16>(exp, g, b, st, U, Ls[0], P, dt, scale, halfdt, hubble);
  else kick_n<32>(exp, g, b, st, U, Ls[0], P, dt, scale, halfdt, hubble);
  return hipGetLastError();
}

double* mg_half_dt(const double* dt, void* work, int nx, int ny, int nz, hipStream_t st) {
  Lvl Ls[kMgMaxLevels];
  int nl;
  double* parts;
  levels_in(work, nx, ny, nz, 1.0, Ls, nl, parts);
  double* slot = parts + kRedParts + 8;
  hipLaunchKernelGGL(mg_scale_scalar, dim3(1), dim3(64), 0, st, dt, slot, 0.5);
  return slot;
}

namespace {

// One V(nu1, nu2) cycle on the levels Ls (level 0 holds f and the initial phi).
void vcycle(const Lvl* Ls, int nl, int nu1, int nu2, hipStream_t st) {
  // rows of n cells: workgroups of up to 256 lanes along x, gx of them per
  // (y, z) row (block_row maps them to rows)
  auto rows = [](int n, int ny, int nz, dim3& g, dim3& blk, int& gx) {
    const int bs = n >= 256 ? 256 : (n + 63) / 64 * 64;
    blk = dim3(bs);
    gx = (n + bs - 1) / bs;
    g = dim3(unsigned(gx), unsigned(ny), unsigned(nz));
  };
  auto smooth = [&](const Lvl& L, int sweeps) {
    dim3 g, blk;
    int gx;
    rows(L.nx / 2, L.ny, L.nz, g, blk, gx);
    for (int s = 0; s < sweeps; s++)
      for (int color = 0; color < 2; color++) hipLaunchKernelGGL(mg_rbgs, g, blk, 0, st, L, color, gx);
  };
  for (int l = 0; l < nl - 1; l++) {
    smooth(Ls[l], nu1);
    dim3 g, blk;
    int gx;
    rows(Ls[l + 1].nx, Ls[l + 1].ny, Ls[l + 1].nz, g, blk, gx);
    hipLaunchKernelGGL(mg_restrict, g, blk, 0, st, Ls[l], Ls[l + 1], gx);
  }
  hipLaunchKernelGGL(mg_coarse_solve, dim3(1), dim3(kCoarseThreads), 0, st, Ls[nl - 1]);
  for (int l = nl - 2; l >= 0; l--) {
    dim3 g, blk;
    int gx;
    rows(Ls[l + 1].nx, Ls[l + 1].ny, Ls[l + 1].nz, g, blk, gx);  // coarse cells
    hipLaunchKernelGGL(mg_prolong_add, g, blk, 0, st, Ls[l + 1], Ls[l], gx);
    smooth(Ls[l], nu2);
  }
}

}  // namespace

hipError_t mg_vcycle_blocks(const DevPlan& P, int nx, int ny, int nz, double h, const double* f_blocks,
                            double* x_padded, int nu1, int nu2, void* work, hipStream_t st) {
  Lvl Ls[kMgMaxLevels];
  int nl;
  double* parts;
  levels_in(work, nx, ny, nz, h, Ls, nl, parts);
  if (P.N != 8 && P.N != 16 && P.N != 32) return hipErrorInvalidValue;
  gather_n<3>(P, f_blocks, nullptr, 0.0, nullptr, Ls[0], st);
  vcycle(Ls, nl, nu1, nu2, st);
  const int64_t nb = P.nleaf * int64_t(P.N) * P.N * P.N;
  const dim3 g(grid_for(nb, 256)), b(256);
  if (P.N == 8) hipLaunchKernelGGL(mg_scatter_padded<8>, g, b, 0, st, Ls[0], P, x_padded);
  else if (P.N == 16) hipLaunchKernelGGL(mg_scatter_padded<16>, g, b, 0, st, Ls[0], P, x_padded);
  else hipLaunchKernelGGL(mg_scatter_padded<32>, g, b, 0, st, Ls[0], P, x_padded);
  return hipGetLastError();
}

hipError_t mg_solve(const DevPlan& P, int nx, int ny, int nz, double h, const double* f_blocks, const double* U,
                    double fpg, double* phi_blocks, int ncycles, int nu1, int nu2, double* resid, void* work,
                    hipStream_t st) {
  Lvl Ls[kMgMaxLevels];
  int nl;
  double* parts;
  levels_in(work, nx, ny, nz, h, Ls, nl, parts);
  double* scal = parts + kRedParts;  // [0] mean of f, [1] mean of phi
  const int64_t n0 = int64_t(nx) * ny * nz;
  const int64_t nb = P.nleaf * int64_t(P.N) * P.N * P.N;
  const dim3 b(256);
  if (P.N != 8 && P.N != 16 && P.N != 32) return hipErrorInvalidValue;
  if (f_blocks) gather_n<0>(P, f_blocks, nullptr, 0.0, phi_blocks, Ls[0], st);
  else gather_n<1>(P, nullptr, U, fpg, phi_blocks, Ls[0], st);
  hipLaunchKernelGGL(mg_sum_parts<0>, dim3(kRedParts), dim3(kRedBlock), 0, st, Ls[0].f, Ls[0], n0, parts);
  hipLaunchKernelGGL(mg_sum_final<0>, dim3(1), dim3(kRedBlock), 0, st, parts, 1.0 / double(n0), scal);
  hipLaunchKernelGGL(mg_sub_mean, dim3(grid_for(n0, 256)), b, 0, st, Ls[0].f, n0, scal);
  auto norm = [&](int c) {
    if (!resid) return;
    hipLaunchKernelGGL(mg_sum_parts<1>, dim3(kRedParts), dim3(kRedBlock), 0, st, nullptr, Ls[0], n0, parts);
    hipLaunchKernelGGL(mg_sum_final<1>, dim3(1), dim3(kRedBlock), 0, st, parts, 1.0, resid + c);
  };
  norm(0);
  for (int c = 0; c < ncycles; c++) {
    vcycle(Ls, nl, nu1, nu2, st);
    norm(c + 1);
  }
  hipLaunchKernelGGL(mg_sum_parts<0>, dim3(kRedParts), dim3(kRedBlock), 0, st, Ls[0].phi, Ls[0], n0, parts);
  hipLaunchKernelGGL(mg_sum_final<0>, dim3(1), dim3(kRedBlock), 0, st, parts, 1.0 / double(n0), scal + 1);
  switch (P.N) {
    case 8: hipLaunchKernelGGL(mg_scatter<8>, dim3(grid_for(nb, 256)), b, 0, st, Ls[0], P, scal + 1, phi_blocks); break;
    case 16: hipLaunchKernelGGL(mg_scatter<16>, dim3(grid_for(nb, 256)), b, 0, st, Ls[0], P, scal + 1, phi_blocks); break;
    default: hipLaunchKernelGGL(mg_scatter<32>, dim3(grid_for(nb, 256)), b, 0, st, Ls[0], P, scal + 1, phi_blocks); break;
  }
  return hipGetLastError();
}

}  // namespace amr
