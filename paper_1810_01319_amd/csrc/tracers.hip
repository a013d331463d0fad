// tracers.hip -- tracer particles on the leaves (Sec. II-B: Lagrangian
// particles live on Blocks, are stored in fixed-size batches and move between
// Blocks; Sec. III: the blast workload carries tracers).
//
// Positions are in level-0 cell units (X in [0, Rx N)), so a particle's
// level-l cell is floor(X 2^l) and wrapping adds or subtracts an integer
// extent exactly.  Storage per leaf: `capacity` slots, a multiple of the batch
// of kTracerBatch; slots 0 .. count-1 hold particles.  One workgroup handles
// one batch of one leaf.
//
// Step: drift each particle with the trilinear interpolation of the cell
// velocities u = m (1/rho) of the refreshed start-of-step state,
// X += (dt u) (Rx N), wrap periodic axes or remove particles leaving through
// an outflow face; find the leaf holding the new position among the leaf
// itself and its 26 neighbours; then write every particle to its leaf in the
// output set: those that stay keep their order, arrivals are appended.
#include <hip/hip_runtime.h>

#include "ghost.hpp"
#include "tracers.hpp"

namespace amr {
namespace {

constexpr int G = kGhost;
constexpr int B = kTracerBatch;

__device__ __forceinline__ int batch_rank(bool pred, int* wave_cnt, int* total) {
  // exclusive rank of this lane among the workgroup's lanes with pred, in
  // lane order; *total receives the count (uses wave_cnt[B / 64])
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long m = __ballot(pred);
  if (lane == 0) wave_cnt[wv] = __popcll(m);
  __syncthreads();
  int before = 0, all = 0;
  for (int w = 0; w < B / 64; w++) {
    const int c = wave_cnt[w];
    before += w < wv ? c : 0;
    all += c;
  }
  *total = all;
  return before + __popcll(m & ((1ull << lane) - 1ull));
}

template <int N>
__global__ void __launch_bounds__(B) tracer_drift(const double* __restrict__ U, const double* __restrict__ dtv,
                                                  DevPlan P, TracerDev T) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  const int64_t s = blockIdx.x / T.nbatch;
  const int b = int(blockIdx.x - s * T.nbatch);
  const int n = T.count_in[s];
  if (b * B >= n) return;  // uniform over the workgroup
  const int slot = b * B + threadIdx.x;
  const bool live = slot < n;
  const BlockInfo bi = P.blocks[s];
  const InstParams& ip = P.inst[bi.inst];
  const int l = bi.level;
  const int key[3] = {bi.i, bi.j, bi.k};
  const int64_t at = s * T.cap + slot;
  int dest = -1;
  int removed = 0, lost = 0;
  bool inside = true;  // a particle outside its leaf (bad input) is dropped as lost, never interpolated
  double X[3] = {0, 0, 0};
  if (live) {
    X[0] = T.pos_in[at];
    X[1] = T.pos_in[T.plane + at];
    X[2] = T.pos_in[2 * T.plane + at];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      const double d = floor(ldexp(X[a], l)) - (double)((int64_t)key[a] * N);
      inside = inside && d >= 0.0 && d < (double)N;
    }
    if (!inside) lost = 1;
  }
  if (live && inside) {
    // trilinear weights and the 8 cells around X
    int i0[3];
    double w[3][2];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      const double sa = (ldexp(X[a], l) - (double)((int64_t)key[a] * N)) - 0.5;
      const double fl = floor(sa);
      i0[a] = (int)fl + G;
      const double f = sa - fl;
      w[a][0] = 1.0 - f;
      w[a][1] = f;
    }
    const double* Bk = U + s * P.nf * M3;
    double c[3][2][2][2];
#pragma unroll
    for (int dz = 0; dz < 2; dz++)
#pragma unroll
      for (int dy = 0; dy < 2; dy++)
#pragma unroll
        for (int dx = 0; dx < 2; dx++) {
          const int64_t o = (int64_t(i0[2] + dz) * M + (i0[1] + dy)) * M + (i0[0] + dx);
          const double ir = 1.0 / Bk[o];
#pragma unroll
          for (int d = 0; d < 3; d++) c[d][dz][dy][dx] = Bk[(1 + d) * M3 + o] * ir;
        }
    const double dt = dtv[bi.inst];
    const double n0 = (double)((int64_t)ip.root[0] * N);
    bool out = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const double z0 = (c[d][0][0][0] * w[0][0] + c[d][0][0][1] * w[0][1]) * w[1][0] +
                        (c[d][0][1][0] * w[0][0] + c[d][0][1][1] * w[0][1]) * w[1][1];
      const double z1 = (c[d][1][0][0] * w[0][0] + c[d][1][0][1] * w[0][1]) * w[1][0] +
                        (c[d][1][1][0] * w[0][0] + c[d][1][1][1] * w[0][1]) * w[1][1];
      const double v = z0 * w[2][0] + z1 * w[2][1];
      const double E = (double)((int64_t)ip.root[d] * N);
      double x = X[d] + (dt * v) * n0;
      if (ip.bc[d] == AMR_BC_PERIODIC_DEV) {
        if (x < 0.0) x += E;
        if (x >= E) x -= E;
      } else if (x < 0.0 || x >= E) {
        out = true;
      }
      X[d] = x;
    }
    if (out) {
      removed = 1;
    } else {
      // the leaf holding X: this one or a neighbour (a particle moves less
      // than a cell per step)
      int o[3];
      bool far = false;
#pragma unroll
      for (int a = 0; a < 3; a++) {
        const int64_t El = ((int64_t)ip.root[a] * N) << l;
        int64_t d = (int64_t)floor(ldexp(X[a], l)) - (int64_t)key[a] * N;
        if (d < -1) d += El;  // wrapped across the periodic seam
        if (d > N) d -= El;
        o[a] = d < 0 ? -1 : (d >= N ? 1 : 0);
        far = far || d < -1 || d > N;
      }
      if (far) {
        lost = 1;
      } else if (o[0] == 0 && o[1] == 0 && o[2] == 0) {
        dest = int(s);
      } else {
        const Nbr e = P.nbr[27 * s + (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)];
        if (e.kind == NBR_FINE) {
          int ch = 0;
#pragma unroll
          for (int a = 0; a < 3; a++) ch |= int(((int64_t)floor(ldexp(X[a], l + 1)) / N) & 1) << a;
          dest = P.fine[8 * int64_t(e.id) + ch];
        } else {
          dest = e.id;
        }
      }
      T.pos_in[at] = X[0];
      T.pos_in[T.plane + at] = X[1];
      T.pos_in[2 * T.plane + at] = X[2];
    }
  }
  if (live) T.dest[at] = dest;  // -1: removed or lost
  __shared__ int wave_cnt[B / 64];
  int stay = 0;
  (void)batch_rank(live && dest == int(s), wave_cnt, &stay);
  if (threadIdx.x == 0) {
    T.stay_batch[s * T.nbatch + b] = stay;
    if (stay) atomicAdd(&T.stay[s], stay);
  }
  const unsigned long long rm = __ballot(removed != 0), ls = __ballot(lost != 0);
  if ((threadIdx.x & 63) == 0) {
    if (rm) atomicAdd(&T.flags[TRACER_REMOVED], (unsigned long long)__popcll(rm));
    if (ls) atomicAdd(&T.flags[TRACER_LOST], (unsigned long long)__popcll(ls));
  }
}

__global__ void __launch_bounds__(B) tracer_scatter(TracerDev T) {
  const int64_t s = blockIdx.x / T.nbatch;
  const int b = int(blockIdx.x - s * T.nbatch);
  const int n = T.count_in[s];
  if (b * B >= n) return;  // uniform over the workgroup
  const int slot = b * B + threadIdx.x;
  const bool live = slot < n;
  const int64_t at = s * T.cap + slot;
  const int dest = live ? T.dest[at] : -1;
  // stayers keep their order: batches before this one, then lanes before this one
  __shared__ int base;
  __shared__ int wave_cnt[B / 64];
  if (threadIdx.x == 0) {
    int sum = 0;
    for (int q = 0; q < b; q++) sum += T.stay_batch[s * T.nbatch + q];
    base = sum;
  }
  int total = 0;
  const int rank = batch_rank(live && dest == int(s), wave_cnt, &total);  // synchronises: base is set
  if (!live || dest < 0) return;
  int64_t to;
  if (dest == int(s)) {
    to = base + rank;
  } else {
    const int k = atomicAdd(&T.arrive[dest], 1);
    to = int64_t(T.stay[dest]) + k;
    if (to >= T.cap) {
      atomicAdd(&T.flags[TRACER_OVERFLOW], 1ull);
      return;
    }
  }
  const int64_t d = int64_t(dest) * T.cap + to;
  T.pos_out[d] = T.pos_in[at];
  T.pos_out[T.plane_out + d] = T.pos_in[T.plane + at];
  T.pos_out[2 * T.plane_out + d] = T.pos_in[2 * T.plane + at];
  T.id_out[d] = T.id_in[at];
}

// After a remesh: the particles of old leaf s go to the leaf that kept it, to
// the child holding their position, or to the merged parent.
__global__ void __launch_bounds__(B) tracer_relocate(DevPlan P, TracerDev T) {
  const int64_t s = blockIdx.x / T.nbatch;
  const int b = int(blockIdx.x - s * T.nbatch);
  const int n = T.count_in[s];
  const int slot = b * B + threadIdx.x;
  if (slot >= n) return;
  const int64_t at = s * T.cap + slot;
  const Reloc r = P.reloc[s];
  const double X[3] = {T.pos_in[at], T.pos_in[T.plane + at], T.pos_in[2 * T.plane + at]};
  int dest = r.id;
  if (r.kind == RELOC_SPLIT) {
    const int32_t* ch = P.reloc_child + 8 * int64_t(r.id);
    const int lc = P.blocks[ch[0]].level;
    int c = 0;
#pragma unroll
    for (int a = 0; a < 3; a++) c |= int(((int64_t)floor(ldexp(X[a], lc)) / P.N) & 1) << a;
    dest = ch[c];
  }
  const int k = atomicAdd(&T.arrive[dest], 1);
  if (k >= T.cap) {
    atomicAdd(&T.flags[TRACER_OVERFLOW], 1ull);
    return;
  }
  const int64_t d = int64_t(dest) * T.cap + k;
  T.pos_out[d] = X[0];
  T.pos_out[T.plane_out + d] = X[1];
  T.pos_out[2 * T.plane_out + d] = X[2];
  T.id_out[d] = T.id_in[at];
}

__global__ void tracer_counts(TracerDev T, int64_t nleaf) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= nleaf) return;
  const int64_t c = int64_t(T.stay[s]) + T.arrive[s];
  T.count_out[s] = int32_t(c < T.cap ? c : T.cap);
  T.stay[s] = 0;  // ready for the next advance
  T.arrive[s] = 0;
}

__global__ void tracer_zero_flags(TracerDev T) {
  if (threadIdx.x < TRACER_NFLAGS) T.flags[threadIdx.x] = 0ull;
}

}  // namespace

hipError_t launch_tracers_advance(const DevPlan& P, const double* U, const double* dt, const TracerDev& T,
                                  hipStream_t st) {
  if (P.nleaf == 0) return hipSuccess;
  const dim3 g(static_cast<unsigned>(P.nleaf * T.nbatch)), b(B);
  switch (P.N) {
    case 8: hipLaunchKernelGGL(tracer_drift<8>, g, b, 0, st, U, dt, P, T); break;
    case 16: hipLaunchKernelGGL(tracer_drift<16>, g, b, 0, st, U, dt, P, T); break;
    case 32: hipLaunchKernelGGL(tracer_drift<32>, g, b, 0, st, U, dt, P, T); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(tracer_scatter, g, b, 0, st, T);
  hipLaunchKernelGGL(tracer_counts, dim3(static_cast<unsigned>((P.nleaf + 255) / 256)), dim3(256), 0, st, T,
                     P.nleaf);
  return hipGetLastError();
}

hipError_t launch_tracers_relocate(const DevPlan& P, int64_t old_nleaf, const TracerDev& T, hipStream_t st) {
  if (old_nleaf > 0)
    hipLaunchKernelGGL(tracer_relocate, dim3(static_cast<unsigned>(old_nleaf * T.nbatch)), dim3(B), 0, st, P, T);
  if (P.nleaf > 0)
    hipLaunchKernelGGL(tracer_counts, dim3(static_cast<unsigned>((P.nleaf + 255) / 256)), dim3(256), 0, st, T,
                       P.nleaf);
  return hipGetLastError();
}

hipError_t launch_tracer_zero_flags(const TracerDev& T, hipStream_t st) {
  hipLaunchKernelGGL(tracer_zero_flags, dim3(1), dim3(64), 0, st, T);
  return hipGetLastError();
}

}  // namespace amr
