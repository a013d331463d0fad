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

#include "expansion_cell.hpp"
#include "kernels.hpp"
#include "ppm_core.hpp"

namespace amr {
namespace {

constexpr int G = kGhost;

__global__ void scale_dt_kernel(const double* __restrict__ dt, double a, const double* __restrict__ a_dev,
                                double* __restrict__ dte, int64_t ninst) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m < ninst) dte[m] = dt[m] / (a_dev ? *a_dev : a);
}

// Flat matter + Lambda expansion (radiation neglected): from
// (adot / a)^2 = H0^2 (om / a^3 + ol) with a(0) = 0,
//   a(t) = (om / ol)^(1/3) sinh(3/2 sqrt(ol) H0 t)^(2/3)   (ol > 0),
//   a(t) = (3/2 H0 t)^(2/3)                                 (ol = 0).
__device__ double cosmo_a(double H0, double om, double ol, double t) {
  if (ol > 0.0) return cbrt(om / ol) * pow(sinh(1.5 * sqrt(ol) * H0 * t), 2.0 / 3.0);
  return pow(1.5 * H0 * t, 2.0 / 3.0);
}

__global__ void cosmology_kernel(int stage, double H0, double om, double ol, const double* __restrict__ dt,
                                 double* __restrict__ cs) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double t = cs[0];
  if (stage == 0) {
    cs[1] = cosmo_a(H0, om, ol, t);
    return;
  }
  const double d = dt[0];
  const double am = cosmo_a(H0, om, ol, t + 0.5 * d);
  cs[2] = am;
  cs[3] = H0 * sqrt(om / (am * am * am) + ol);
  cs[0] = t + d;
}

// One thread per active cell.
template <int N>
__global__ void __launch_bounds__(256) expansion_kernel(double* __restrict__ U, const double* __restrict__ dtv,
                                                        double hubble, const double* __restrict__ hubble_dev,
                                                        DevPlan P) {
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
  const double c = (0.5 * dtv[bi.inst]) * (hubble_dev ? *hubble_dev : hubble);
  double* const B = U + int64_t(s) * P.nf * M3 + (int64_t(z + G) * M + (y + G)) * M + (x + G);
  const bool de = P.nf == kFieldsDE;
  const double rho = B[0];
  double mx = B[M3], my = B[2 * M3], mz = B[3 * M3], E = B[4 * M3], ge = de ? B[5 * M3] : 0.0;
  const unsigned nfl = expansion_cell(ip, c, de, rho, mx, my, mz, E, ge);
  B[M3] = mx;
  B[2 * M3] = my;
  B[3 * M3] = mz;
  B[4 * M3] = E;
  if (de) B[5 * M3] = ge;
  if (nfl) atomicAdd(P.counters, (unsigned long long)nfl);
}

// Transpose of expansion_kernel: lam holds dL/dU after the sources on entry
// and dL/dU before them on exit, at the state U they were applied to (NF = 5,
// or 6 with the dual-energy field).  One thread per active cell.
template <int N, int NF>
__global__ void __launch_bounds__(256) expansion_adjoint_kernel(const double* __restrict__ U,
                                                                double* __restrict__ lam,
                                                                const double* __restrict__ dtv, double hubble,
                                                                DevPlan P) {
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
  const int64_t o = int64_t(s) * NF * M3 + (int64_t(z + G) * M + (y + G)) * M + (x + G);
  const double* const B = U + o;
  double* const L = lam + o;
  double lr = L[0], lmx = L[M3], lmy = L[2 * M3], lmz = L[3 * M3], lE = L[4 * M3];
  expansion_cell_vjp(ip, c, B[0], B[M3], B[2 * M3], B[3 * M3], B[4 * M3], lr, lmx, lmy, lmz, lE);
  L[0] = lr;
  L[M3] = lmx;
  L[2 * M3] = lmy;
  L[3 * M3] = lmz;
  L[4 * M3] = lE;
  if constexpr (NF == kFieldsDE) {
    double lge = L[5 * M3];
    expansion_ge_vjp(ip, c, B[5 * M3], lge);
    L[5 * M3] = lge;
  }
}

template <int N>
hipError_t expansion_adjoint_n(const DevPlan& P, const double* U, double* lam, const double* dt, double hubble,
                               hipStream_t st) {
  const int64_t n = P.nleaf * int64_t(N) * N * N;
  if (n > 0) {
    if (P.nf == kFieldsDE)
      hipLaunchKernelGGL((expansion_adjoint_kernel<N, kFieldsDE>), dim3(static_cast<unsigned>((n + 255) / 256)),
                         dim3(256), 0, st, U, lam, dt, hubble, P);
    else
      hipLaunchKernelGGL((expansion_adjoint_kernel<N, kFields>), dim3(static_cast<unsigned>((n + 255) / 256)),
                         dim3(256), 0, st, U, lam, dt, hubble, P);
  }
  return hipGetLastError();
}

template <int N>
hipError_t expansion_n(const DevPlan& P, double* U, const double* dt, double hubble, const double* hubble_dev,
                       hipStream_t st) {
  const int64_t n = P.nleaf * int64_t(N) * N * N;
  if (n > 0)
    hipLaunchKernelGGL(expansion_kernel<N>, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, U, dt,
                       hubble, hubble_dev, P);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_scale_dt(const DevPlan& P, const double* dt, double a, hipStream_t st, const double* a_dev) {
  if (P.ninst > 0)
    hipLaunchKernelGGL(scale_dt_kernel, dim3(static_cast<unsigned>((P.ninst + 63) / 64)), dim3(64), 0, st, dt, a,
                       a_dev, P.dte, P.ninst);
  return hipGetLastError();
}

hipError_t launch_expansion(const DevPlan& P, double* U, const double* dt, double hubble, hipStream_t st,
                            const double* hubble_dev) {
  switch (P.N) {
    case 8: return expansion_n<8>(P, U, dt, hubble, hubble_dev, st);
    case 16: return expansion_n<16>(P, U, dt, hubble, hubble_dev, st);
    case 32: return expansion_n<32>(P, U, dt, hubble, hubble_dev, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_expansion_adjoint(const DevPlan& P, const double* U, double* lam, const double* dt, double hubble,
                                   hipStream_t st) {
  switch (P.N) {
    case 8: return expansion_adjoint_n<8>(P, U, lam, dt, hubble, st);
    case 16: return expansion_adjoint_n<16>(P, U, lam, dt, hubble, st);
    case 32: return expansion_adjoint_n<32>(P, U, lam, dt, hubble, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cosmology(int stage, double H0, double om, double ol, const double* dt, double* cs,
                            hipStream_t st) {
  hipLaunchKernelGGL(cosmology_kernel, dim3(1), dim3(64), 0, st, stage, H0, om, ol, dt, cs);
  return hipGetLastError();
}

}  // namespace amr
