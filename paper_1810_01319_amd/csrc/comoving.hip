// comoving.hip -- comoving coordinates for the ppm Method (paper Sec. II-C:
// the hydro method supports cosmological comoving expansion terms; the terms
// follow Bryan et al. 1995).  x is the comoving position, v the peculiar
// velocity, a(t) the expansion factor and H = adot / a.  The flux divergence
// carries 1/a, so a comoving step runs the plain refresh, sweeps and reflux
// with dt / a; the CFL dt is (C_cfl * a) * min dx / (max_d |v_d| + c); the
// expansion sources dv/dt = -H v, d(rho e)/dt = -3 (gamma - 1) H rho e (the
// comoving density is unchanged) follow the reflux with Crank-Nicolson
// factors at the step's mid time, c = (dt / 2) H:
//   m' = m fv,   fv = (1 - c) / (1 + c)
//   ie' = ie fe, fe = (1 - 3 (gamma - 1) c) / (1 + 3 (gamma - 1) c)
//   E' = E + ((ie' - ie) + ke (fv fv - 1))
// (H = 0 leaves a cell bit for bit); where the source lowered the internal
// energy below the pressure floor it is raised to it and counted.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "ppm_core.hpp"

namespace amr {
namespace {

constexpr int G = kGhost;

__global__ void scale_dt_kernel(const double* __restrict__ dt, double a, double* __restrict__ dte, int64_t ninst) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m < ninst) dte[m] = dt[m] / a;
}

// One thread per active cell.
template <int N>
__global__ void __launch_bounds__(256) expansion_kernel(double* __restrict__ U, const double* __restrict__ dtv,
                                                        double hubble, DevPlan P) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int x = q % N, y = (q / N) % N, z = q / (N * N);
  const BlockInfo bi = P.blocks[s];
  const InstParams ip = P.inst[bi.inst];
  const double c = (0.5 * dtv[bi.inst]) * hubble;
  const double g3 = 3.0 * ip.gm1;
  const double fv = (1.0 - c) / (1.0 + c);
  const double fe = (1.0 - g3 * c) / (1.0 + g3 * c);
  double* const B = U + int64_t(s) * P.nf * M3 + (int64_t(z + G) * M + (y + G)) * M + (x + G);
  const double rho = B[0], mx = B[M3], my = B[2 * M3], mz = B[3 * M3], E = B[4 * M3];
  const double ir = rcp_pos(rho);
  const double u = mx * ir, v = my * ir, w = mz * ir;
  const double ke = (0.5 * rho) * ((u * u + v * v) + w * w);
  const double ie = E - ke;
  double ie2 = ie * fe;
  const bool fl = ie2 < ie && ip.gm1 * ie2 < ip.p_floor;
  if (fl) ie2 = ip.p_floor * ip.inv_gm1;
  B[M3] = mx * fv;
  B[2 * M3] = my * fv;
  B[3 * M3] = mz * fv;
  B[4 * M3] = E + ((ie2 - ie) + ke * (fv * fv - 1.0));
  unsigned long long nfl = fl ? 1ull : 0ull;
  if (P.nf == kFieldsDE) {  // the dual-energy field: the same factor and floor rule
    const double ge = B[5 * M3];
    double ge2 = ge * fe;
    if (ge2 < ge && ip.gm1 * ge2 < ip.p_floor) {
      ge2 = ip.p_floor * ip.inv_gm1;
      nfl++;
    }
    B[5 * M3] = ge2;
  }
  if (nfl) atomicAdd(P.counters, nfl);
}

template <int N>
hipError_t expansion_n(const DevPlan& P, double* U, const double* dt, double hubble, hipStream_t st) {
  const int64_t n = P.nleaf * int64_t(N) * N * N;
  if (n > 0)
    hipLaunchKernelGGL(expansion_kernel<N>, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, U, dt,
                       hubble, P);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_scale_dt(const DevPlan& P, const double* dt, double a, hipStream_t st) {
  if (P.ninst > 0)
    hipLaunchKernelGGL(scale_dt_kernel, dim3(static_cast<unsigned>((P.ninst + 63) / 64)), dim3(64), 0, st, dt, a,
                       P.dte, P.ninst);
  return hipGetLastError();
}

hipError_t launch_expansion(const DevPlan& P, double* U, const double* dt, double hubble, hipStream_t st) {
  switch (P.N) {
    case 8: return expansion_n<8>(P, U, dt, hubble, st);
    case 16: return expansion_n<16>(P, U, dt, hubble, st);
    case 32: return expansion_n<32>(P, U, dt, hubble, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace amr
