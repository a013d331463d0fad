// kernels.hip -- gfx950 kernels of one AMR hydro step.
//
// Paper Sec. II-B (ghost refresh of width 3 for the 5 conserved fields,
// Restrict / Prolong across 2:1 jumps) and Sec. II-C (the PPM Method).
// Built with -ffp-contract=off: no fused multiply-add, so every formula
// rounds exactly as written; FP64 '/' and sqrt are IEEE correctly rounded
// on gfx950.  min/max are selects (a < b ? a : b).
//
// Storage: per leaf 5 fields of M^3 doubles, M = N + 6, x fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.hpp"
#include "ppm_core.hpp"
#include "ghost.hpp"
#include "xcd.hpp"

namespace amr {

namespace {

constexpr int G = kGhost;


// dx at level l: cubic cells, x extent 1.
__device__ __forceinline__ double level_dx(const InstParams& ip, int N, int l) {
  return 1.0 / (double)((int64_t)ip.root[0] * N << l);
}

// ---------------------------------------------------------------------------
// Ghost refresh
// ---------------------------------------------------------------------------

// Phase 1: same-level copies (incl. outflow clamps) and restriction.  On
// large meshes the workgroups go to the XCDs in contiguous ranges (a leaf's
// ghost cells and its neighbours' in one L2) and the ghost cells are written
// with non-temporal stores (the sweeps read them from HBM either way); on
// small ones in hardware order, which spreads the leaves of a refined region,
// and their restriction work, over all XCDs, with ordinary stores.
// LARGE: the large-mesh instantiation (the two store kinds must be separate
// kernels: under a run-time branch the compiler merges them into one plain
// store).
template <int N, int NF, bool LARGE>
__global__ void __launch_bounds__(256) refresh_phase1(double* __restrict__ U, DevPlan P) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int GC = M * M * M - N * N * N;
  const int64_t t = int64_t(LARGE ? xcd_block() : blockIdx.x) * blockDim.x + threadIdx.x;
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
  double* dst = U + int64_t(s) * NF * M3 + (int64_t(c) * M + b) * M + a;
  if (e.kind == NBR_COPY) {
    const BlockInfo sb = P.blocks[e.id];
    const int la = px - sb.i * N + G, lb = py - sb.j * N + G, lc = pz - sb.k * N + G;
    const double* src = U + int64_t(e.id) * NF * M3 + (int64_t(lc) * M + lb) * M + la;
#pragma unroll
    for (int f = 0; f < NF; f++) {
      if constexpr (LARGE) __builtin_nontemporal_store(src[f * M3], dst + f * M3);
      else dst[f * M3] = src[f * M3];
    }
  } else {
    // mean of the 8 children, summed x fastest then y then z
    const int qx = 2 * px, qy = 2 * py, qz = 2 * pz;
    const int cidx = ((qx / N) & 1) + 2 * ((qy / N) & 1) + 4 * ((qz / N) & 1);
    const int fs = P.fine[8 * int64_t(e.id) + cidx];
    const int la = qx % N + G, lb = qy % N + G, lc = qz % N + G;
    const double* src = U + int64_t(fs) * NF * M3 + (int64_t(lc) * M + lb) * M + la;
#pragma unroll
    for (int f = 0; f < NF; f++) {
      const double* q = src + f * M3;
      const double v0 = q[0], v1 = q[1], v2 = q[M], v3 = q[M + 1];
      const double v4 = q[M * M], v5 = q[M * M + 1], v6 = q[M * M + M], v7 = q[M * M + M + 1];
      const double m = (((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7))) * 0.125;
      if constexpr (LARGE) __builtin_nontemporal_store(m, dst + f * M3);
      else dst[f * M3] = m;
    }
  }
}

// Phase 2: limited linear prolongation from the coarser leaf, whose active
// and phase-1 ghost cells are complete, over the ghost regions (faces,
// edges, corners) whose neighbour position a coarser leaf covers.  One
// thread per field of a group of ghost cells that share a coarse parent (up
// to 2 x 2 x 2): the parent's stencil is loaded and its slopes computed
// once, then each cell of the group takes its own offset.  One launch covers
// every region, in leaf order, so that a leaf's face, edge and corner
// regions run together and share the coarse cells and output lines they
// touch in L2; each wave of the task table runs once per field (fields
// innermost).  Each task takes whole waves, so the task, its leaves and
// their instance are wave-uniform: scalar loads, off the latency chain of
// the stencil loads.
// LIN: unlimited central slopes 0.5 (u(+1) - u(-1)) (the composite Poisson
// operator's interpolation).
template <int N, int NF, bool LIN, int K>
__device__ __forceinline__ void phase2_group(double* __restrict__ U, const DevPlan& P, int s, int code, int r,
                                             int f) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  if (r >= P2Region<N, K>::GROUPS) return;
  // group -> its cells' padded ranges along x, y, z (x fastest)
  const int cl[3] = {code % 3, (code / 3) % 3, code / 9};
  int first[3], cnt[3], j = r;
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const int ng = cl[d] == 1 ? N / 2 : 2;  // a power of two
    p2_group<N>(cl[d], j & (ng - 1), first[d], cnt[d]);
    j /= ng;
  }
  const Nbr e = P.nbr[27 * int64_t(s) + code];  // a coarser leaf, by construction
  const BlockInfo bi = P.blocks[s];
  const InstParams ip = P.inst[bi.inst];  // by value: read once, before the stores
  const int l = bi.level;
  const BlockInfo cb = P.blocks[e.id];
  // the parent (the same for every cell of the group)
  const int px0 = bc_index<N>(ip, l, 0, bi.i * N + first[0] - G);
  const int py0 = bc_index<N>(ip, l, 1, bi.j * N + first[1] - G);
  const int pz0 = bc_index<N>(ip, l, 2, bi.k * N + first[2] - G);
  const int la = (px0 >> 1) - cb.i * N + G, lb = (py0 >> 1) - cb.j * N + G, lc = (pz0 >> 1) - cb.k * N + G;
  const double* q = U + (int64_t(e.id) * NF + f) * M3 + (int64_t(lc) * M + lb) * M + la;
  const double u0 = q[0];
  double sx, sy, sz;
  if (LIN) {
    sx = 0.5 * (q[1] - q[-1]);
    sy = 0.5 * (q[M] - q[-M]);
    sz = 0.5 * (q[M * M] - q[-M * M]);
  } else {
    sx = minmod(q[1] - u0, u0 - q[-1]);
    sy = minmod(q[M] - u0, u0 - q[-M]);
    sz = minmod(q[M * M] - u0, u0 - q[-M * M]);
  }
  double* const dst0 = U + (int64_t(s) * NF + f) * M3;
  for (int dc = 0; dc < cnt[2]; dc++) {
    const int c = first[2] + dc;
    const double oz = (bc_index<N>(ip, l, 2, bi.k * N + c - G) & 1) ? 0.25 : -0.25;
    for (int db = 0; db < cnt[1]; db++) {
      const int b = first[1] + db;
      const double oy = (bc_index<N>(ip, l, 1, bi.j * N + b - G) & 1) ? 0.25 : -0.25;
      for (int da = 0; da < cnt[0]; da++) {
        const int a = first[0] + da;
        const double ox = (bc_index<N>(ip, l, 0, bi.i * N + a - G) & 1) ? 0.25 : -0.25;
        dst0[(int64_t(c) * M + b) * M + a] = ((u0 + ox * sx) + oy * sy) + oz * sz;
      }
    }
  }
}

template <int N, int NF, bool LIN>
__global__ void __launch_bounds__(256) refresh_phase2(double* __restrict__ U, DevPlan P) {
  const unsigned wf = xcd_block() * (blockDim.x >> 6) + unsigned(__builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)));
  const unsigned w = wf / unsigned(NF);  // table wave, then the field
  const int f = int(wf - w * unsigned(NF));
  if (w >= unsigned(P.np2w)) return;
  const int e = P.p2wave[w];
  const int row = e >> kP2SubBits;
  const int r = (e & ((1 << kP2SubBits) - 1)) * 64 + int(threadIdx.x & 63u);
  const int s = P.p2task[2 * int64_t(row)], code = P.p2task[2 * int64_t(row) + 1];
  // the region's kind from its direction: a face has two interior axes
  const int nin = (code % 3 == 1) + ((code / 3) % 3 == 1) + (code / 9 == 1);
  if (nin == 2) phase2_group<N, NF, LIN, 0>(U, P, s, code, r, f);
  else if (nin == 1) phase2_group<N, NF, LIN, 1>(U, P, s, code, r, f);
  else phase2_group<N, NF, LIN, 2>(U, P, s, code, r, f);
}

// ---------------------------------------------------------------------------
// CFL reduction
// ---------------------------------------------------------------------------

template <int N, int NF>
__global__ void __launch_bounds__(256) cfl_kernel(const double* __restrict__ U, DevPlan P, int chunks) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int s = blockIdx.x / chunks;
  const int ch = blockIdx.x - s * chunks;
  const BlockInfo bi = P.blocks[s];
  const InstParams& ip = P.inst[bi.inst];
  const double dx = level_dx(ip, N, bi.level);
  const double* B = U + int64_t(s) * NF * M3;
  const int per = N3 / chunks;
  double best = __builtin_huge_val();
  for (int q = ch * per + threadIdx.x; q < (ch + 1) * per; q += blockDim.x) {
    const int x = q % N, y = (q / N) % N, z = q / (N * N);
    const int64_t o = (int64_t(z + G) * M + (y + G)) * M + (x + G);
    const double rho = B[o];
    const double ir = rcp_pos(rho);
    const double u = B[o + M3] * ir, v = B[o + 2 * M3] * ir, w = B[o + 3 * M3] * ir;
    double ge = 0.0;
    if constexpr (NF == kFieldsDE) ge = B[o + 5 * M3];
    double p = gas_pressure<NF == kFieldsDE>(ip, rho, u, v, w, B[o + 4 * M3], ge);
    p = p < ip.p_floor ? ip.p_floor : p;
    const double cs = sqrt_pos((ip.gamma * p) * ir);
    const double vm = sel_max(sel_max(fabs(u), fabs(v)), fabs(w));
    const double dtc = dx / (vm + cs);
    best = dtc < best ? dtc : best;
  }
  // wave64 then workgroup minimum; the minimum is exact in any order
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(best, off, 64);
    best = o < best ? o : best;
  }
  __shared__ double red[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < int(blockDim.x >> 6); i++) best = red[i] < best ? red[i] : best;
    // positive doubles order like their bit patterns
    atomicMin(&P.acc[bi.inst], (unsigned long long)__double_as_longlong(best));
  }
}

// Floor-reset counter bookkeeping, one lane: mode 0 copies the counter to
// *mark, mode 1 replaces *mark by the resets since (counter - *mark), mode 2
// copies *mark back into the counter.
__global__ void floor_mark(DevPlan P, unsigned long long* __restrict__ mark, int mode) {
  if (blockIdx.x * blockDim.x + threadIdx.x != 0) return;
  if (mode == 0) mark[threadIdx.x] = P.counters[threadIdx.x];
  else if (mode == 1) mark[threadIdx.x] = P.counters[threadIdx.x] - mark[threadIdx.x];
  else P.counters[threadIdx.x] = mark[threadIdx.x];
}

// a_dev (nullable): the expansion factor on the device, in place of a
__global__ void cfl_finalize(DevPlan P, double* __restrict__ dt, double a, const double* __restrict__ a_dev) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= P.ninst) return;
  const double mn = __longlong_as_double((long long)P.acc[m]);
  const double av = a_dev ? *a_dev : a;
  dt[m] = (P.inst[m].cfl * av) * mn;  // a = 1 leaves cfl * mn bit for bit
  P.acc[m] = 0x7FF0000000000000ull;
}

// Signal speed max_d |u_d| + c of one cell from its conserved values
// (momenta in x, y, z order), in exactly the CFL kernel's arithmetic; ir =
// 1/rho.  A run of steps keeps each leaf's maximum: correctly rounded
// division is monotone, so dx / (leaf maximum) is the leaf's minimum of
// dx / speed bit for bit, and the per-cell division is saved.
template <bool DE = false>
__device__ __forceinline__ double cfl_speed(const InstParams& ip, double rho, double ir, double mx, double my,
                                            double mz, double E, double ge = 0.0) {
  const double u = mx * ir, v = my * ir, w = mz * ir;
  double p = gas_pressure<DE>(ip, rho, u, v, w, E, ge);
  p = p < ip.p_floor ? ip.p_floor : p;
  const double cs = sqrt_pos((ip.gamma * p) * ir);
  const double vm = sel_max(sel_max(fabs(u), fabs(v)), fabs(w));
  return vm + cs;
}

// dt of each instance from the per-leaf maximum signal speeds a run of steps
// accumulated, over the whole grid: one thread per leaf takes its maximum
// (and resets the slots to 0) and dx / speed, and the minimum goes into the
// instance's accumulator (one atomic per wave whose leaves share an
// instance, else lane by lane; positive doubles order like their bit
// patterns, so the minimum is exact in any order); cfl_finalize then forms
// C_cfl times it.
__global__ void __launch_bounds__(256) cfl_leaf_min(DevPlan P) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  unsigned long long v = 0x7FF0000000000000ull;  // +inf
  int inst = -1;
  if (s < P.nleaf) {
    const BlockInfo bi = P.blocks[s];
    inst = bi.inst;
    unsigned long long sb = 0ull;
    for (int k = 0; k < kCflSlots; k++) {
      const unsigned long long x = P.lacc[s * kCflSlots + k];
      sb = x > sb ? x : sb;
      P.lacc[s * kCflSlots + k] = 0ull;
    }
    const double t = level_dx(P.inst[inst], P.N, bi.level) / __longlong_as_double((long long)sb);
    v = (unsigned long long)__double_as_longlong(t);
  }
  // lane 0 holds the wave's first leaf: a wave without leaves has inst -1 everywhere
  const int i0 = __shfl(inst, 0, 64);
  if (i0 < 0) return;
  if (__ballot(inst == i0 || inst < 0) == __ballot(1)) {
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(v, off, 64);
      v = o < v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) atomicMin(&P.acc[i0], v);
  } else if (inst >= 0) {
    atomicMin(&P.acc[inst], v);
  }
}

// Whether the reflux will still correct cell (x, y, z) of a leaf whose
// corrected faces are the bits 2 d + side of rflx.
__device__ __forceinline__ bool in_reflux_layer(int rflx, int N, int x, int y, int z) {
  const int q[3] = {x, y, z};
  bool in = false;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    in = in || (((rflx >> (2 * a)) & 1) && q[a] == G) || (((rflx >> (2 * a + 1)) & 1) && q[a] == G + N - 1);
  }
  return in;
}

// Maximum over a full wave, then one atomic per wave (non-negative doubles
// order like their bit patterns); partial waves add lane by lane.
__device__ __forceinline__ void cfl_commit(unsigned long long* acc, double best) {
  if (__ballot(1) == ~0ull) {
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(best, off, 64);
      best = o > best ? o : best;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(acc, (unsigned long long)__double_as_longlong(best));
  } else {
    atomicMax(acc, (unsigned long long)__double_as_longlong(best));
  }
}

// ---------------------------------------------------------------------------
// PPM sweep: one lane walks one pencil along the sweep axis with a sliding
// register window; the next cell is prefetched one step ahead, and each cell
// is updated three cells behind the read front (the stencil of a cell update
// is 7 cells wide).  The conserved values of the last three cells read wait
// in a per-lane ring in LDS (3 cells x NF fields, lane-minor, dynamic shared
// memory of 3 NF blockDim.x doubles), so the update takes them from there
// instead of reading HBM a second time.
// ---------------------------------------------------------------------------

constexpr int kWalkLanes = 256;  // workgroup size bound of the walk kernels

// cfl_next (the last sweep of a step in a run of steps): every updated cell
// that no reflux will change adds its CFL candidate for the next step to the
// instance's accumulator.
template <int N, int DIR, bool OOP, int NF>
__device__ __forceinline__ void sweep_walk_body(const double* Uin, double* Uout, const double* __restrict__ dtv,
                                                const DevPlan& P, int loA, int nA, int loB, int nB, int cfl_next,
                                                double* __restrict__ ring) {
  constexpr bool DE = NF == kFieldsDE;  // dual-energy field rho e (field 5)
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int A = DIR == 0 ? 1 : 0;
  constexpr int B = DIR == 2 ? 1 : 2;
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;  // velocity roles
  constexpr int SD = DIR == 0 ? 1 : (DIR == 1 ? M : M * M);
  constexpr int SA = A == 0 ? 1 : (A == 1 ? M : M * M);
  constexpr int SB = B == 0 ? 1 : (B == 1 ? M : M * M);
  // waves never straddle two leaves: the leaf index is wave-uniform, so the
  // leaf's and the instance's parameters are scalar loads
  const int npen = nA * nB;
  const unsigned wpl = unsigned(npen + 63) / 64u;
  const unsigned w = xcd_block() * (blockDim.x >> 6) + unsigned(__builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)));
  const int s = int(w / wpl);
  const int pp = int(w - unsigned(s) * wpl) * 64 + int(threadIdx.x & 63u);
  if (s >= P.nleaf || pp >= npen) return;
  const int iA = loA + pp % nA, iB = loB + pp / nA;
  const BlockInfo bi = P.blocks[s];
  const InstParams ip = P.inst[bi.inst];  // by value: read once, before any store
  const double dxl = level_dx(ip, N, bi.level);
  const double nu = dtv[bi.inst] / dxl;
  double cfl_best = 0.0;  // maximum signal speed (cfl_next)
  const int64_t boff = int64_t(s) * NF * M3 + int64_t(iA) * SA + int64_t(iB) * SB;
  const double* const pr_ = Uin + boff;
  const double* const pn_ = pr_ + (1 + DIR) * M3;
  const double* const p1_ = pr_ + (1 + T1) * M3;
  const double* const p2_ = pr_ + (1 + T2) * M3;
  const double* const pe_ = pr_ + 4 * M3;
  double* const qr_ = Uout + boff;
  double* const qn_ = qr_ + (1 + DIR) * M3;
  double* const q1_ = qr_ + (1 + T1) * M3;
  double* const q2_ = qr_ + (1 + T2) * M3;
  double* const qe_ = qr_ + 4 * M3;
  const double* const pg_ = pr_ + 5 * M3;  // rho e: dereferenced only with DE
  double* const qg_ = qr_ + 5 * M3;
  const bool faces_act = iA >= G && iA < G + N && iB >= G && iB < G + N;
  int slot_lo = -1, slot_hi = -1;
  if (faces_act) {
    slot_lo = P.faceslot[6 * int64_t(s) + 2 * DIR];
    slot_hi = P.faceslot[6 * int64_t(s) + 2 * DIR + 1];
  }
  const int64_t face_off = int64_t(iB - G) * N + (iA - G);
  const double gm1 = ip.gm1, pfl = ip.p_floor, rfl = ip.rho_floor, sixth = ip.sixth;

  if (OOP) {  // cells the sweep does not update pass through
#pragma unroll
    for (int k = 0; k < 2 * G; k++) {
      const int64_t o = int64_t(k < G ? k : N + k) * SD;
      qr_[o] = pr_[o]; qn_[o] = pn_[o]; q1_[o] = p1_[o]; q2_[o] = p2_[o]; qe_[o] = pe_[o];
      if constexpr (DE) qg_[o] = pg_[o];
    }
  }

  // windows: rho, v, w over cells t-2..t; u over t-3..t; p over t-4..t;
  // c and 1/rho over t-2..t
  double rw[3], vw[3], ww[3], uw[4], pw[5], cw[3], iw[3];
  double dl[5][2];   // slopes of cells t-2, t-1
  double fold[5];    // face value at (t-3)+1/2
  double WLp[5];     // left state at (t-3)+1/2 from cell t-3
  double Fp[NF];     // flux at (t-4)+1/2
  double ugp = 0.0;  // Godunov velocity at (t-4)+1/2 (DE)
  unsigned nfl = 0;
  // prefetch cell 0
  double nx0 = pr_[0], nx1 = pn_[0], nx2 = p1_[0], nx3 = p2_[0], nx4 = pe_[0], nx5 = 0.0;
  if constexpr (DE) nx5 = pg_[0];
  // One cell of the walk.  The walk is split into a head (cells 0..5: no
  // update yet; the lower coarse-fine face flux), a body in which every cell
  // issues the same loads and stores (so that waiting for the prefetched cell
  // never waits for the previous cell's stores) and the last cell (the upper
  // face flux).
  // ring slot of cell c: c mod 3, rotating with the walk; field stride L
  const int L = int(blockDim.x);
  double* const rl = ring + threadIdx.x;
  int rs = 0;
  auto cell = [&](const int c, auto phase) __attribute__((always_inline)) {
    constexpr int PH = decltype(phase)::value;
    double h0 = 0, h1 = 0, h2 = 0, h3 = 0, h4 = 0, h5 = 0;
    double* const slot = rl + rs * (NF * L);
    if (PH > 0) {  // the cell updated here, c-3: its values left the ring's slot c mod 3
      h0 = slot[0]; h1 = slot[L]; h2 = slot[2 * L]; h3 = slot[3 * L]; h4 = slot[4 * L];
      if constexpr (DE) h5 = slot[5 * L];
    }
    const double U0 = nx0, U1 = nx1, U2 = nx2, U3 = nx3, U4 = nx4, U5 = nx5;
    slot[0] = U0; slot[L] = U1; slot[2 * L] = U2; slot[3 * L] = U3; slot[4 * L] = U4;
    if constexpr (DE) slot[5 * L] = U5;
    rs = rs == 2 ? 0 : rs + 1;
    if (PH < 2) {
      const int64_t o = int64_t(c + 1) * SD;
      nx0 = pr_[o]; nx1 = pn_[o]; nx2 = p1_[o]; nx3 = p2_[o]; nx4 = pe_[o];
      if constexpr (DE) nx5 = pg_[o];
    }
    // primitives of cell c
    const double ir = rcp_pos(U0);
    const double u = U1 * ir, v = U2 * ir, w = U3 * ir;
    double p = gas_pressure<DE>(ip, U0, u, v, w, U4, U5);
    p = p < pfl ? pfl : p;
    const double cs = sqrt_pos((ip.gamma * p) * ir);
    rw[0] = rw[1]; rw[1] = rw[2]; rw[2] = U0;
    vw[0] = vw[1]; vw[1] = vw[2]; vw[2] = v;
    ww[0] = ww[1]; ww[1] = ww[2]; ww[2] = w;
    uw[0] = uw[1]; uw[1] = uw[2]; uw[2] = uw[3]; uw[3] = u;
    pw[0] = pw[1]; pw[1] = pw[2]; pw[2] = pw[3]; pw[3] = pw[4]; pw[4] = p;
    cw[0] = cw[1]; cw[1] = cw[2]; cw[2] = cs;
    iw[0] = iw[1]; iw[1] = iw[2]; iw[2] = ir;
    if (PH == 0 && c < 2) return;
    // slope of cell c-1
#pragma unroll
    for (int q = 0; q < 5; q++) dl[q][0] = dl[q][1];
    dl[0][1] = mc_slope(rw[0], rw[1], rw[2]);
    dl[1][1] = mc_slope(uw[1], uw[2], uw[3]);
    dl[2][1] = mc_slope(vw[0], vw[1], vw[2]);
    dl[3][1] = mc_slope(ww[0], ww[1], ww[2]);
    dl[4][1] = mc_slope(pw[2], pw[3], pw[4]);
    if (PH == 0 && c < 3) return;
    // face value at (c-2)+1/2
    double fnew[5];
    fnew[0] = 0.5 * (rw[0] + rw[1]) - (dl[0][1] - dl[0][0]) * sixth;
    fnew[1] = 0.5 * (uw[1] + uw[2]) - (dl[1][1] - dl[1][0]) * sixth;
    fnew[2] = 0.5 * (vw[0] + vw[1]) - (dl[2][1] - dl[2][0]) * sixth;
    fnew[3] = 0.5 * (ww[0] + ww[1]) - (dl[3][1] - dl[3][0]) * sixth;
    fnew[4] = 0.5 * (pw[2] + pw[3]) - (dl[4][1] - dl[4][0]) * sixth;
    if (PH > 0 || c >= 4) {
      // cell j = c-2: flattening, parabolas, tracing
      const double pp1 = pw[3], pm1 = pw[1];
      const double dp1 = pp1 - pm1;
      const double pmin = pp1 < pm1 ? pp1 : pm1;
      const bool shock = (fabs(dp1) > 0.33 * pmin) && (uw[0] - uw[2] > 0.0);
      const double dp2 = pw[4] - pw[0];
      const double r = (dp2 != 0.0) ? dp1 / dp2 : 0.0;
      double ft = 10.0 * (r - 0.75);
      ft = ft < 1.0 ? ft : 1.0;
      ft = ft > 0.0 ? ft : 0.0;
      const double f = shock ? ft : 0.0;
      Par pa[5];
      pa[0] = parabola(rw[0], fold[0], fnew[0], f, sixth);
      pa[1] = parabola(uw[1], fold[1], fnew[1], f, sixth);
      pa[2] = parabola(vw[0], fold[2], fnew[2], f, sixth);
      pa[3] = parabola(ww[0], fold[3], fnew[3], f, sixth);
      pa[4] = parabola(pw[2], fold[4], fnew[4], f, sixth);
      double WL[5], WR[5];
      trace(ip, rw[0], uw[1], cw[0], iw[0], pa, nu, WL, WR);
      if (PH > 0 || c >= 5) {
        // flux at (c-3)+1/2 from cell c-3's right edge and cell c-2's left
        double F[NF], ugn = 0.0;
        riemann_flux<DE>(ip, WLp, WR, F, &ugn);
        if (PH == 0 && slot_lo >= 0) {  // c = G+2: lower face of the active cells
          double* fo = P.faces + int64_t(slot_lo) * NF * N * N + face_off;
          fo[0] = F[0]; fo[(1 + DIR) * N * N] = F[1]; fo[(1 + T1) * N * N] = F[2];
          fo[(1 + T2) * N * N] = F[3]; fo[4 * N * N] = F[4];
          if constexpr (DE) fo[5 * N * N] = F[5];
        }
        if (PH == 2 && slot_hi >= 0) {  // c = N+G+2: upper face
          double* fo = P.faces + int64_t(slot_hi) * NF * N * N + face_off;
          fo[0] = F[0]; fo[(1 + DIR) * N * N] = F[1]; fo[(1 + T1) * N * N] = F[2];
          fo[(1 + T2) * N * N] = F[3]; fo[4 * N * N] = F[4];
          if constexpr (DE) fo[5 * N * N] = F[5];
        }
        if (PH > 0) {
          // conservative update of cell c-3, then the floors
          const int64_t o = int64_t(c - 3) * SD;
          double r0 = h0 - nu * (F[0] - Fp[0]);
          const double m1 = h1 - nu * (F[1] - Fp[1]);
          const double m2 = h2 - nu * (F[2] - Fp[2]);
          const double m3 = h3 - nu * (F[3] - Fp[3]);
          double e = h4 - nu * (F[4] - Fp[4]);
          if (r0 < rfl) { r0 = rfl; nfl++; }
          const double jr = rcp_pos(r0);
          const double a1 = m1 * jr, a2 = m2 * jr, a3 = m3 * jr;
          const double ke = (0.5 * r0) * ((a1 * a1 + a2 * a2) + a3 * a3);
          const double pn = gm1 * (e - ke);
          if (pn < pfl) { e = pfl * ip.inv_gm1 + ke; nfl++; }
          qr_[o] = r0; qn_[o] = m1; q1_[o] = m2; q2_[o] = m3; qe_[o] = e;
          double ge = 0.0;
          if constexpr (DE) {
            // rho e: its flux difference, the work of cell c-3's pressure
            // (pw[1]) on the Godunov velocities, then the resynchronisation
            // from E where E - ke > eta2 E and the floor
            ge = h5 - nu * (F[5] - Fp[5]);
            ge = ge - nu * (pw[1] * (ugn - ugp));
            const double ie = e - ke;
            if (ie > ip.eta2 * e) ge = ie;
            if (gm1 * ge < pfl) { ge = pfl * ip.inv_gm1; nfl++; }
            qg_[o] = ge;
          }
          if (cfl_next) {
            int q[3];
            q[DIR] = c - 3;
            q[A] = iA;
            q[B] = iB;
            if (!in_reflux_layer(bi.rflx, N, q[0], q[1], q[2])) {
              double mv[3];
              mv[DIR] = m1;
              mv[T1] = m2;
              mv[T2] = m3;
              const double t = cfl_speed<DE>(ip, r0, jr, mv[0], mv[1], mv[2], e, ge);
              cfl_best = t > cfl_best ? t : cfl_best;
            }
          }
        }
#pragma unroll
        for (int q = 0; q < NF; q++) Fp[q] = F[q];
        ugp = ugn;
      }
#pragma unroll
      for (int q = 0; q < 5; q++) WLp[q] = WL[q];
    }
#pragma unroll
    for (int q = 0; q < 5; q++) fold[q] = fnew[q];
  };
  static_assert(G == 3, "the walk's head covers cells 0..2G-1");
  for (int c = 0; c < 2 * G; c++) cell(c, std::integral_constant<int, 0>{});
  // one full wait on entry to the body: its loop then starts from the same
  // outstanding-memory state on every pass
  __builtin_amdgcn_s_waitcnt(0);
  for (int c = 2 * G; c < M - 1; c++) cell(c, std::integral_constant<int, 1>{});
  cell(M - 1, std::integral_constant<int, 2>{});
  if (nfl) atomicAdd(P.counters, (unsigned long long)nfl);
  if (cfl_next) cfl_commit(&P.lacc[int64_t(s) * kCflSlots + ((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kCflSlots)], cfl_best);
}

template <int N, int DIR, int NF>
__global__ void __launch_bounds__(kWalkLanes) sweep_kernel(double* __restrict__ U, const double* __restrict__ dtv,
                                                           DevPlan P, int loA, int nA, int loB, int nB, int cfl_next) {
  extern __shared__ double walk_ring[];
  sweep_walk_body<N, DIR, false, NF>(U, U, dtv, P, loA, nA, loB, nB, cfl_next, walk_ring);
}

// Out of place: every cell of the swept pencils is written to Uout (updated
// or passed through); Uin is not modified.
template <int N, int DIR, int NF>
__global__ void __launch_bounds__(kWalkLanes) sweep_kernel_oop(const double* __restrict__ Uin,
                                                               double* __restrict__ Uout,
                                                               const double* __restrict__ dtv, DevPlan P, int loA,
                                                               int nA, int loB, int nB) {
  extern __shared__ double walk_ring[];
  sweep_walk_body<N, DIR, true, NF>(Uin, Uout, dtv, P, loA, nA, loB, nB, 0, walk_ring);
}

// ---------------------------------------------------------------------------
// PPM sweep, LDS-staged: a workgroup owns a tile of R whole pencils, loaded
// with coalesced accesses (along x a tile is R consecutive rows, contiguous
// unless it spans two z layers; along y or z it is R consecutive x
// positions).  Each thread
// owns one cell of the tile through six stages separated by barriers; its own
// cell's state stays in registers and only neighbour values go through LDS.
// ---------------------------------------------------------------------------

template <int N, int DIR>
struct StagedShape {
  static constexpr int M = N + 2 * G;
  // pencils per tile (measured on gfx950: 3-row tiles run the x sweep 7%
  // faster than 5-row ones at N = 32)
  static constexpr int R = N == 8 ? 9 : (N == 16 ? 11 : (DIR == 0 ? 3 : 5));
  static constexpr int T = R * M;  // cells per tile
  static constexpr int WG = ((T + 63) / 64) * 64;
};

template <int N, int DIR, bool OOP, int NF>
__device__ __forceinline__ void sweep_staged_body(const double* Uin, double* Uout, const double* __restrict__ dtv,
                                                  const DevPlan& P, int loA, int nA, int loB, int nB,
                                                  int cfl_next) {
  constexpr bool DE = NF == kFieldsDE;  // dual-energy field rho e (field 5)
  using S = StagedShape<N, DIR>;
  constexpr int M = S::M, R = S::R, T = S::T;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int A = DIR == 0 ? 1 : 0;
  constexpr int B = DIR == 2 ? 1 : 2;
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
  constexpr int SD = DIR == 0 ? 1 : (DIR == 1 ? M : M * M);
  constexpr int SA = A == 0 ? 1 : (A == 1 ? M : M * M);
  constexpr int SB = B == 0 ? 1 : (B == 1 ? M : M * M);
  constexpr int NS = DIR == 0 ? 1 : R;  // item stride between neighbouring cells
  __shared__ double Ps[5][T];           // primitives
  __shared__ double Xs[5][T];           // slopes, then right states at j-1/2
  __shared__ double Ys[5][T];           // face values at j+1/2, then fluxes
  __shared__ double Fg[DE ? T : 1];     // DE: rho e flux at j+1/2
  __shared__ double Ug[DE ? T : 1];     // DE: Godunov velocity at j+1/2
  // tile -> (leaf, its first pencil): a tile is R consecutive pencils of the
  // leaf's nA x nB plane (numbered along A, then B; the pencils are
  // independent, so a tile may span two B rows and only the leaf's last tile
  // is partial); 32-bit unsigned arithmetic on the uniform tile index (a grid
  // has fewer than 2^32 workgroups)
  const int npen = nA * nB;
  const unsigned tpl = unsigned(npen + R - 1) / unsigned(R);
  const unsigned tile = xcd_block();
  const int s = int(tile / tpl);
  const int i = threadIdx.x;
  const int r = DIR == 0 ? i / M : i % R;
  const int c = DIR == 0 ? i - r * M : i / R;
  const int pp = int(tile - unsigned(s) * tpl) * R + r;
  const bool live = i < T && pp < npen;
  const BlockInfo bi = P.blocks[s];
  const InstParams& ip = P.inst[bi.inst];
  const double nu = dtv[bi.inst] / level_dx(ip, N, bi.level);
  const int iA = loA + pp % nA, iB = loB + pp / nA;
  const int64_t coff = int64_t(s) * NF * M3 + int64_t(iA) * SA + int64_t(iB) * SB + int64_t(c) * SD;
  const double* const cellp = Uin + coff;
  double* const outp = Uout + coff;
  const double gm1 = ip.gm1, pfl = ip.p_floor, rfl = ip.rho_floor, sixth = ip.sixth;

  // A: own cell, primitives
  double U0 = 0, U1 = 0, U2 = 0, U3 = 0, U4 = 0, U5 = 0, q[5] = {0, 0, 0, 0, 0}, cs = 0, ir = 0;
  if (live) {
    U0 = cellp[0];
    U1 = cellp[(1 + DIR) * M3];
    U2 = cellp[(1 + T1) * M3];
    U3 = cellp[(1 + T2) * M3];
    U4 = cellp[4 * M3];
    if constexpr (DE) U5 = cellp[5 * M3];
    ir = rcp_pos(U0);
    q[0] = U0;
    q[1] = U1 * ir;
    q[2] = U2 * ir;
    q[3] = U3 * ir;
    double p = gas_pressure<DE>(ip, U0, q[1], q[2], q[3], U4, U5);
    q[4] = p < pfl ? pfl : p;
    cs = sqrt_pos((ip.gamma * q[4]) * ir);
#pragma unroll
    for (int v = 0; v < 5; v++) Ps[v][i] = q[v];
  }
  __syncthreads();
  // B: limited slopes
  if (live && c >= 1 && c <= M - 2) {
#pragma unroll
    for (int v = 0; v < 5; v++) Xs[v][i] = mc_slope(Ps[v][i - NS], q[v], Ps[v][i + NS]);
  }
  __syncthreads();
  // C: face values at c+1/2
  if (live && c >= 1 && c <= M - 3) {
#pragma unroll
    for (int v = 0; v < 5; v++)
      Ys[v][i] = 0.5 * (q[v] + Ps[v][i + NS]) - (Xs[v][i + NS] - Xs[v][i]) * sixth;
  }
  __syncthreads();
  // D: flattening, parabolas, characteristic tracing
  double WL[5] = {0, 0, 0, 0, 0}, WR[5];
  const bool traced = live && c >= 2 && c <= M - 3;
  if (traced) {
    const double pp1 = Ps[4][i + NS], pm1 = Ps[4][i - NS];
    const double dp1 = pp1 - pm1;
    const double pmin = pp1 < pm1 ? pp1 : pm1;
    const bool shock = (fabs(dp1) > 0.33 * pmin) && (Ps[1][i - NS] - Ps[1][i + NS] > 0.0);
    const double dp2 = Ps[4][i + 2 * NS] - Ps[4][i - 2 * NS];
    const double rr = (dp2 != 0.0) ? dp1 / dp2 : 0.0;
    double ft = 10.0 * (rr - 0.75);
    ft = ft < 1.0 ? ft : 1.0;
    ft = ft > 0.0 ? ft : 0.0;
    const double f = shock ? ft : 0.0;
    Par pa[5];
#pragma unroll
    for (int v = 0; v < 5; v++) pa[v] = parabola(q[v], Ys[v][i - NS], Ys[v][i], f, sixth);
    trace(ip, q[0], q[1], cs, ir, pa, nu, WL, WR);
  }
  __syncthreads();
  if (traced) {
#pragma unroll
    for (int v = 0; v < 5; v++) Xs[v][i] = WR[v];
  }
  __syncthreads();
  // E: Riemann flux at c+1/2
  if (live && c >= 2 && c <= M - 4) {
    double R5[5], F[NF], ugn = 0.0;
#pragma unroll
    for (int v = 0; v < 5; v++) R5[v] = Xs[v][i + NS];
    riemann_flux<DE>(ip, WL, R5, F, &ugn);
#pragma unroll
    for (int v = 0; v < 5; v++) Ys[v][i] = F[v];
    if constexpr (DE) {
      Fg[i] = F[5];
      Ug[i] = ugn;
    }
    const bool faces_act = iA >= G && iA < G + N && iB >= G && iB < G + N;
    if (faces_act && (c == G - 1 || c == N + G - 1)) {
      const int slot = P.faceslot[6 * int64_t(s) + 2 * DIR + (c == G - 1 ? 0 : 1)];
      if (slot >= 0) {
        double* fo = P.faces + int64_t(slot) * NF * N * N + int64_t(iB - G) * N + (iA - G);
        fo[0] = F[0]; fo[(1 + DIR) * N * N] = F[1]; fo[(1 + T1) * N * N] = F[2];
        fo[(1 + T2) * N * N] = F[3]; fo[4 * N * N] = F[4];
        if constexpr (DE) fo[5 * N * N] = F[5];
      }
    }
  }
  __syncthreads();
  // F: conservative update of the active cells, floors
  double cfl_best = 0.0;  // signal speed (cfl_next)
  if (live && c >= G && c < G + N) {
    double r0 = U0 - nu * (Ys[0][i] - Ys[0][i - NS]);
    const double m1 = U1 - nu * (Ys[1][i] - Ys[1][i - NS]);
    const double m2 = U2 - nu * (Ys[2][i] - Ys[2][i - NS]);
    const double m3 = U3 - nu * (Ys[3][i] - Ys[3][i - NS]);
    double e = U4 - nu * (Ys[4][i] - Ys[4][i - NS]);
    unsigned nfl = 0;
    if (r0 < rfl) { r0 = rfl; nfl++; }
    const double jr = rcp_pos(r0);
    const double a1 = m1 * jr, a2 = m2 * jr, a3 = m3 * jr;
    const double ke = (0.5 * r0) * ((a1 * a1 + a2 * a2) + a3 * a3);
    const double pn = gm1 * (e - ke);
    if (pn < pfl) { e = pfl * ip.inv_gm1 + ke; nfl++; }
    outp[0] = r0;
    outp[(1 + DIR) * M3] = m1;
    outp[(1 + T1) * M3] = m2;
    outp[(1 + T2) * M3] = m3;
    outp[4 * M3] = e;
    double ge = 0.0;
    if constexpr (DE) {  // rho e: flux difference, work, resynchronisation, floor (as in the walk)
      ge = U5 - nu * (Fg[i] - Fg[i - NS]);
      ge = ge - nu * (q[4] * (Ug[i] - Ug[i - NS]));
      const double ie = e - ke;
      if (ie > ip.eta2 * e) ge = ie;
      if (gm1 * ge < pfl) { ge = pfl * ip.inv_gm1; nfl++; }
      outp[5 * M3] = ge;
    }
    if (nfl) atomicAdd(P.counters, (unsigned long long)nfl);
    if (cfl_next) {  // the next step's CFL candidate (see the walk)
      int q[3];
      q[DIR] = c;
      q[A] = iA;
      q[B] = iB;
      if (!in_reflux_layer(bi.rflx, N, q[0], q[1], q[2])) {
        double mv[3];
        mv[DIR] = m1;
        mv[T1] = m2;
        mv[T2] = m3;
        cfl_best = cfl_speed<DE>(ip, r0, jr, mv[0], mv[1], mv[2], e, ge);
      }
    }
  } else if (OOP && live) {  // cells the sweep does not update pass through
    outp[0] = U0;
    outp[(1 + DIR) * M3] = U1;
    outp[(1 + T1) * M3] = U2;
    outp[(1 + T2) * M3] = U3;
    outp[4 * M3] = U4;
    if constexpr (DE) outp[5 * M3] = U5;
  }
  if (cfl_next) cfl_commit(&P.lacc[int64_t(s) * kCflSlots + ((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kCflSlots)], cfl_best);
}

template <int N, int DIR, int NF>
__global__ void __launch_bounds__((StagedShape<N, DIR>::WG)) sweep_staged(double* __restrict__ U,
                                                                    const double* __restrict__ dtv, DevPlan P,
                                                                    int loA, int nA, int loB, int nB,
                                                                    int cfl_next) {
  sweep_staged_body<N, DIR, false, NF>(U, U, dtv, P, loA, nA, loB, nB, cfl_next);
}

template <int N, int DIR, int NF>
__global__ void __launch_bounds__((StagedShape<N, DIR>::WG)) sweep_staged_oop(const double* __restrict__ Uin,
                                                                        double* __restrict__ Uout,
                                                                        const double* __restrict__ dtv, DevPlan P,
                                                                        int loA, int nA, int loB, int nB) {
  sweep_staged_body<N, DIR, true, NF>(Uin, Uout, dtv, P, loA, nA, loB, nB, 0);
}

// ---------------------------------------------------------------------------
// Reflux
// ---------------------------------------------------------------------------

template <int N, int DIR, int NF>
__global__ void __launch_bounds__(256) reflux_kernel(double* __restrict__ U, const double* __restrict__ dtv,
                                                     DevPlan P) {
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
  const double nu = dtv[bi.inst] / level_dx(ip, N, bi.level);
  const int hA = tA >= N / 2, hB = tB >= N / 2;
  const int fs = T.slot_f[hA + 2 * hB];
  const int fA = 2 * tA - hA * N, fB = 2 * tB - hB * N;
  const int d = T.side ? N + G - 1 : G;
  double* cellp = U + int64_t(T.leaf) * NF * M3 + int64_t(d) * SD + int64_t(G + tA) * SA + int64_t(G + tB) * SB;
#pragma unroll
  for (int f = 0; f < NF; f++) {
    const double Fc = P.faces[(int64_t(T.slot_c) * NF + f) * N * N + int64_t(tB) * N + tA];
    const double* Q = P.faces + (int64_t(fs) * NF + f) * N * N;
    const double fb = ((Q[fB * N + fA] + Q[fB * N + fA + 1]) + (Q[(fB + 1) * N + fA] + Q[(fB + 1) * N + fA + 1])) * 0.25;
    const double corr = nu * (Fc - fb);
    const double u = cellp[f * M3];
    cellp[f * M3] = T.side ? u + corr : u - corr;
  }
}

// ---------------------------------------------------------------------------
// Remesh: indicator and data migration
// ---------------------------------------------------------------------------

// S_b = max over active cells and axes of |rho(+1) - rho(-1)| / (2 rho); one
// workgroup per leaf, exact maximum.
template <int N>
__global__ void __launch_bounds__(256) indicator_kernel(const double* __restrict__ U, DevPlan P) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int s = blockIdx.x;
  const double* B = U + int64_t(s) * P.nf * M3;
  double best = 0.0;
  for (int q = threadIdx.x; q < N3; q += blockDim.x) {
    const int x = q % N, y = (q / N) % N, z = q / (N * N);
    const int64_t o = (int64_t(z + G) * M + (y + G)) * M + (x + G);
    const double r0 = B[o];
    const double sx = fabs(B[o + 1] - B[o - 1]) / (2.0 * r0);
    const double sy = fabs(B[o + M] - B[o - M]) / (2.0 * r0);
    const double sz = fabs(B[o + M * M] - B[o - M * M]) / (2.0 * r0);
    best = sx > best ? sx : best;
    best = sy > best ? sy : best;
    best = sz > best ? sz : best;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(best, off, 64);
    best = o > best ? o : best;
  }
  __shared__ double red[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < int(blockDim.x >> 6); i++) best = red[i] > best ? red[i] : best;
    P.ind[s] = best;
  }
}

// One thread per active cell of a new leaf: copy, prolong from the old
// parent's refreshed block (the refresh prolongation formula), or restrict
// the 8 old children.
template <int N, int NF>
__global__ void __launch_bounds__(256) migrate_kernel(const double* __restrict__ Uold, double* __restrict__ Unew,
                                                      DevPlan P) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int N3 = N * N * N;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nleaf * N3) return;
  const int s = int(t / N3);
  const int q = int(t - int64_t(s) * N3);
  const int a = q % N, b = (q / N) % N, c = q / (N * N);
  const MigrTask T = P.migr[s];
  double* dst = Unew + int64_t(s) * NF * M3 + (int64_t(c + G) * M + (b + G)) * M + (a + G);
  if (T.kind == MIGR_COPY) {
    const double* src = Uold + int64_t(T.src[0]) * NF * M3 + (int64_t(c + G) * M + (b + G)) * M + (a + G);
#pragma unroll
    for (int f = 0; f < NF; f++) dst[f * M3] = src[f * M3];
  } else if (T.kind == MIGR_PROLONG) {
    const int cx = T.co & 1, cy = (T.co >> 1) & 1, cz = (T.co >> 2) & 1;
    const int la = (cx * N + a) / 2 + G, lb = (cy * N + b) / 2 + G, lc = (cz * N + c) / 2 + G;
    const double ox = (a & 1) ? 0.25 : -0.25, oy = (b & 1) ? 0.25 : -0.25, oz = (c & 1) ? 0.25 : -0.25;
    const double* src = Uold + int64_t(T.src[0]) * NF * M3 + (int64_t(lc) * M + lb) * M + la;
#pragma unroll
    for (int f = 0; f < NF; f++) {
      const double* qq = src + f * M3;
      const double u0 = qq[0];
      const double sx = minmod(qq[1] - u0, u0 - qq[-1]);
      const double sy = minmod(qq[M] - u0, u0 - qq[-M]);
      const double sz = minmod(qq[M * M] - u0, u0 - qq[-M * M]);
      dst[f * M3] = ((u0 + ox * sx) + oy * sy) + oz * sz;
    }
  } else {
    const int fx = 2 * a, fy = 2 * b, fz = 2 * c;
    const int ch = (fx / N) + 2 * (fy / N) + 4 * (fz / N);
    const int la = fx % N + G, lb = fy % N + G, lc = fz % N + G;
    const double* src = Uold + int64_t(T.src[ch]) * NF * M3 + (int64_t(lc) * M + lb) * M + la;
#pragma unroll
    for (int f = 0; f < NF; f++) {
      const double* qq = src + f * M3;
      const double v0 = qq[0], v1 = qq[1], v2 = qq[M], v3 = qq[M + 1];
      const double v4 = qq[M * M], v5 = qq[M * M + 1], v6 = qq[M * M + M], v7 = qq[M * M + M + 1];
      dst[f * M3] = (((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7))) * 0.125;
    }
  }
}

inline unsigned grid_for(int64_t n, int block) { return unsigned((n + block - 1) / block); }

// the phase-2 launch: whole waves per task and field, in leaf order (wave
// indices are 32-bit)
template <int N, int NF, bool LIN>
hipError_t launch_phase2(const DevPlan& P, double* U, int block, hipStream_t st) {
  const int64_t n = P.np2w * NF * 64;  // threads
  if (n >= (int64_t(1) << 32)) return hipErrorInvalidValue;
  if (n > 0) hipLaunchKernelGGL((refresh_phase2<N, NF, LIN>), dim3(grid_for(n, block)), dim3(block), 0, st, U, P);
  return hipSuccess;
}

// dynamic LDS of a walk launch: the per-lane ring of 3 cells x nf fields
inline size_t walk_ring_bytes(int nf, int block) { return size_t(3) * nf * block * sizeof(double); }

template <int N, int NF>
hipError_t refresh_nf(const DevPlan& P, double* U, const LaunchCfg& L, hipStream_t st) {
  constexpr int M = N + 2 * G;
  constexpr int64_t GC = int64_t(M) * M * M - int64_t(N) * N * N;
  if (P.nleaf > 0) {
    const dim3 g(grid_for(P.nleaf * GC, L.refresh_block)), b(L.refresh_block);
    if (P.p1_large) hipLaunchKernelGGL((refresh_phase1<N, NF, true>), g, b, 0, st, U, P);
    else hipLaunchKernelGGL((refresh_phase1<N, NF, false>), g, b, 0, st, U, P);
  }
  if (P.np2 > 0) {
    const hipError_t e = launch_phase2<N, NF, false>(P, U, L.refresh_block, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

template <int N>
hipError_t refresh_n(const DevPlan& P, double* U, const LaunchCfg& L, hipStream_t st) {
  return P.nf == kFieldsDE ? refresh_nf<N, kFieldsDE>(P, U, L, st) : refresh_nf<N, kFields>(P, U, L, st);
}

template <int N>
hipError_t cfl_n(const DevPlan& P, const double* U, double* dt, const LaunchCfg& L, hipStream_t st, double a,
                 const double* a_dev) {
  constexpr int N3 = N * N * N;
  int chunks = N3 / (8 * 256);
  if (chunks < 1) chunks = 1;
  if (P.nleaf > 0) {
    if (P.nf == kFieldsDE)
      hipLaunchKernelGGL((cfl_kernel<N, kFieldsDE>), dim3(unsigned(P.nleaf * chunks)), dim3(256), 0, st, U, P, chunks);
    else
      hipLaunchKernelGGL((cfl_kernel<N, kFields>), dim3(unsigned(P.nleaf * chunks)), dim3(256), 0, st, U, P, chunks);
  }
  hipLaunchKernelGGL(cfl_finalize, dim3(grid_for(P.ninst, 64)), dim3(64), 0, st, P, dt, a, a_dev);
  return hipGetLastError();
}

template <int N, int DIR, int NF>
hipError_t sweep_ndf(const DevPlan& P, const double* Uin, double* Uout, const double* dt, const int swept[3],
                     const LaunchCfg& L, hipStream_t st, int cfl_next) {
  constexpr int M = N + 2 * G;
  constexpr int A = DIR == 0 ? 1 : 0;
  constexpr int B = DIR == 2 ? 1 : 2;
  const int loA = swept[A] ? G : 0, nA = swept[A] ? N : M;
  const int loB = swept[B] ? G : 0, nB = swept[B] ? N : M;
  if (P.nleaf == 0) return hipSuccess;
  const bool oop = Uin != Uout;
  if (L.sweep_mode[DIR] == 1) {
    using S = StagedShape<N, DIR>;
    const dim3 g(static_cast<unsigned>(P.nleaf * ((int64_t(nA) * nB + S::R - 1) / S::R))), b(S::WG);
    if (oop)
      hipLaunchKernelGGL((sweep_staged_oop<N, DIR, NF>), g, b, 0, st, Uin, Uout, dt, P, loA, nA, loB, nB);
    else
      hipLaunchKernelGGL((sweep_staged<N, DIR, NF>), g, b, 0, st, Uout, dt, P, loA, nA, loB, nB, cfl_next);
  } else {
    const int64_t n = P.nleaf * ((int64_t(nA) * nB + 63) / 64) * 64;  // whole waves per leaf
    const dim3 g(grid_for(n, L.sweep_block)), b(L.sweep_block);
    const size_t ring = walk_ring_bytes(NF, L.sweep_block);
    if (oop)
      hipLaunchKernelGGL((sweep_kernel_oop<N, DIR, NF>), g, b, ring, st, Uin, Uout, dt, P, loA, nA, loB, nB);
    else
      hipLaunchKernelGGL((sweep_kernel<N, DIR, NF>), g, b, ring, st, Uout, dt, P, loA, nA, loB, nB, cfl_next);
  }
  return hipGetLastError();
}

template <int N, int DIR>
hipError_t sweep_nd(const DevPlan& P, const double* Uin, double* Uout, const double* dt, const int swept[3],
                    const LaunchCfg& L, hipStream_t st, int cfl_next) {
  if (P.nf == kFieldsDE) return sweep_ndf<N, DIR, kFieldsDE>(P, Uin, Uout, dt, swept, L, st, cfl_next);
  return sweep_ndf<N, DIR, kFields>(P, Uin, Uout, dt, swept, L, st, cfl_next);
}

template <int N>
hipError_t sweep_n(const DevPlan& P, const double* Uin, double* Uout, const double* dt, int dir, const int swept[3],
                   const LaunchCfg& L, hipStream_t st, int cfl_next) {
  if (dir == 0) return sweep_nd<N, 0>(P, Uin, Uout, dt, swept, L, st, cfl_next);
  if (dir == 1) return sweep_nd<N, 1>(P, Uin, Uout, dt, swept, L, st, cfl_next);
  return sweep_nd<N, 2>(P, Uin, Uout, dt, swept, L, st, cfl_next);
}

// The next step's CFL candidates of the cells the reflux corrected (one
// thread per cell of each task's face layer; cells on two corrected faces
// are counted twice, which a minimum ignores).
template <int N, int DIR, int NF>
__global__ void __launch_bounds__(256) reflux_cfl_kernel(const double* __restrict__ U, DevPlan P) {
  constexpr int M = N + 2 * G;
  constexpr int64_t M3 = int64_t(M) * M * M;
  constexpr int A = DIR == 0 ? 1 : 0;
  constexpr int B = DIR == 2 ? 1 : 2;
  constexpr int SD = DIR == 0 ? 1 : (DIR == 1 ? M : M * M);
  constexpr int SA = A == 0 ? 1 : (A == 1 ? M : M * M);
  constexpr int SB = B == 0 ? 1 : (B == 1 ? M : M * M);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P.nreflux[DIR] * N * N) return;  // N * N is a multiple of 64: whole waves
  const int k = int(t / (N * N));
  const int r = int(t - int64_t(k) * N * N);
  const RefluxTask T = P.reflux[DIR][k];
  const BlockInfo bi = P.blocks[T.leaf];
  const InstParams ip = P.inst[bi.inst];
  const int d = T.side ? N + G - 1 : G;
  const double* B0 = U + int64_t(T.leaf) * NF * M3 + int64_t(d) * SD + int64_t(G + r % N) * SA +
                     int64_t(G + r / N) * SB;
  const double rho = B0[0];
  double ge = 0.0;
  if constexpr (NF == kFieldsDE) ge = B0[5 * M3];
  const double c = cfl_speed<NF == kFieldsDE>(ip, rho, rcp_pos(rho), B0[M3], B0[2 * M3], B0[3 * M3], B0[4 * M3], ge);
  cfl_commit(&P.lacc[int64_t(T.leaf) * kCflSlots + ((t >> 6) % kCflSlots)], c);
}

template <int N, int NF>
hipError_t reflux_cfl_nf(const DevPlan& P, const double* U, hipStream_t st) {
  for (int d = 0; d < 3; d++) {
    const int64_t n = P.nreflux[d] * N * N;
    if (n == 0) continue;
    const dim3 g(grid_for(n, 256)), b(256);
    if (d == 0) hipLaunchKernelGGL((reflux_cfl_kernel<N, 0, NF>), g, b, 0, st, U, P);
    else if (d == 1) hipLaunchKernelGGL((reflux_cfl_kernel<N, 1, NF>), g, b, 0, st, U, P);
    else hipLaunchKernelGGL((reflux_cfl_kernel<N, 2, NF>), g, b, 0, st, U, P);
  }
  return hipGetLastError();
}

template <int N>
hipError_t reflux_cfl_n(const DevPlan& P, const double* U, hipStream_t st) {
  return P.nf == kFieldsDE ? reflux_cfl_nf<N, kFieldsDE>(P, U, st) : reflux_cfl_nf<N, kFields>(P, U, st);
}

template <int N, int NF>
hipError_t reflux_nf(const DevPlan& P, double* U, const double* dt, int dir, const LaunchCfg& L, hipStream_t st) {
  const int64_t n = P.nreflux[dir] * N * N;
  if (n == 0) return hipSuccess;
  const dim3 g(grid_for(n, L.reflux_block)), b(L.reflux_block);
  if (dir == 0) hipLaunchKernelGGL((reflux_kernel<N, 0, NF>), g, b, 0, st, U, dt, P);
  else if (dir == 1) hipLaunchKernelGGL((reflux_kernel<N, 1, NF>), g, b, 0, st, U, dt, P);
  else hipLaunchKernelGGL((reflux_kernel<N, 2, NF>), g, b, 0, st, U, dt, P);
  return hipGetLastError();
}

template <int N>
hipError_t reflux_n(const DevPlan& P, double* U, const double* dt, int dir, const LaunchCfg& L, hipStream_t st) {
  return P.nf == kFieldsDE ? reflux_nf<N, kFieldsDE>(P, U, dt, dir, L, st) : reflux_nf<N, kFields>(P, U, dt, dir, L, st);
}

}  // namespace


template <int N>
hipError_t refresh_scalar_n(const DevPlan& P, double* x, hipStream_t st) {
  constexpr int M = N + 2 * G;
  constexpr int64_t GC = int64_t(M) * M * M - int64_t(N) * N * N;
  if (P.nleaf > 0 && P.p1_large)
    hipLaunchKernelGGL((refresh_phase1<N, 1, true>), dim3(grid_for(P.nleaf * GC, 256)), dim3(256), 0, st, x, P);
  else if (P.nleaf > 0)
    hipLaunchKernelGGL((refresh_phase1<N, 1, false>), dim3(grid_for(P.nleaf * GC, 256)), dim3(256), 0, st, x, P);
  if (P.np2 > 0) {
    const hipError_t e = launch_phase2<N, 1, true>(P, x, 256, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_refresh_scalar(const DevPlan& P, double* x, hipStream_t st) {
  switch (P.N) {
    case 8: return refresh_scalar_n<8>(P, x, st);
    case 16: return refresh_scalar_n<16>(P, x, st);
    case 32: return refresh_scalar_n<32>(P, x, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_refresh(const DevPlan& P, double* U, const LaunchCfg& L, hipStream_t st) {
  switch (P.N) {
    case 8: return refresh_n<8>(P, U, L, st);
    case 16: return refresh_n<16>(P, U, L, st);
    case 32: return refresh_n<32>(P, U, L, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cfl(const DevPlan& P, const double* U, double* dt, const LaunchCfg& L, hipStream_t st, double a,
                      const double* a_dev) {
  switch (P.N) {
    case 8: return cfl_n<8>(P, U, dt, L, st, a, a_dev);
    case 16: return cfl_n<16>(P, U, dt, L, st, a, a_dev);
    case 32: return cfl_n<32>(P, U, dt, L, st, a, a_dev);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sweep(const DevPlan& P, double* U, const double* dt, int dir, const int swept[3],
                        const LaunchCfg& L, hipStream_t st) {
  return launch_sweep_oop(P, U, U, dt, dir, swept, L, st);
}

hipError_t launch_sweep_oop(const DevPlan& P, const double* Uin, double* Uout, const double* dt, int dir,
                            const int swept[3], const LaunchCfg& L, hipStream_t st, int cfl_next) {
  if (cfl_next && Uin != Uout) return hipErrorInvalidValue;  // only the in-place sweeps feed the next CFL
  switch (P.N) {
    case 8: return sweep_n<8>(P, Uin, Uout, dt, dir, swept, L, st, cfl_next);
    case 16: return sweep_n<16>(P, Uin, Uout, dt, dir, swept, L, st, cfl_next);
    case 32: return sweep_n<32>(P, Uin, Uout, dt, dir, swept, L, st, cfl_next);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reflux_cfl(const DevPlan& P, const double* U, hipStream_t st) {
  switch (P.N) {
    case 8: return reflux_cfl_n<8>(P, U, st);
    case 16: return reflux_cfl_n<16>(P, U, st);
    case 32: return reflux_cfl_n<32>(P, U, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cfl_finalize(const DevPlan& P, double* dt, hipStream_t st) {
  if (P.ninst <= 0) return hipSuccess;
  if (P.nleaf > 0) hipLaunchKernelGGL(cfl_leaf_min, dim3(grid_for(P.nleaf, 256)), dim3(256), 0, st, P);
  hipLaunchKernelGGL(cfl_finalize, dim3(grid_for(P.ninst, 64)), dim3(64), 0, st, P, dt, 1.0, nullptr);
  return hipGetLastError();
}

hipError_t launch_floor_mark(const DevPlan& P, unsigned long long* mark, int mode, hipStream_t st) {
  hipLaunchKernelGGL(floor_mark, dim3(1), dim3(64), 0, st, P, mark, mode);
  return hipGetLastError();
}

// Self-test of rcp_pos and sqrt_pos against the IEEE operations: operand i
// has a random mantissa and an exponent uniform over [-767, 1022], drawn
// from the splitmix64 hash of seed + i (Steele, Lea and Flood 2014); the
// first operands of seed 0 are 1, 2^-767, 1.5 * 2^1021 and 2^1022.
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) arith_check_kernel(uint64_t seed, int64_t n,
                                                         unsigned long long* __restrict__ bad) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = seed + uint64_t(i);
  const uint64_t h = splitmix64(k), g = splitmix64(k ^ 0x5DEECE66Dull);
  const int64_t ex = -767 + int64_t(g % 1790u);
  double x = __longlong_as_double((long long)((uint64_t(ex + 1023) << 52) | (h & ((1ull << 52) - 1))));
  if (k == 0) x = 1.0;
  if (k == 1) x = 0x1p-767;
  if (k == 2) x = 0x1.8p+1021;
  if (k == 3) x = 0x1p+1022;
  const double r = rcp_pos(x), q = 1.0 / x, a = sqrt_pos(x), b = sqrt(x);
  const unsigned nr = __double_as_longlong(r) != __double_as_longlong(q);
  const unsigned ns = __double_as_longlong(a) != __double_as_longlong(b);
  if (nr) atomicAdd(&bad[0], 1ull);
  if (ns) atomicAdd(&bad[1], 1ull);
}

hipError_t launch_arith_check(uint64_t seed, int64_t n, unsigned long long* bad, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(arith_check_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, seed, n, bad);
  return hipGetLastError();
}

hipError_t launch_indicator(const DevPlan& P, const double* U, hipStream_t st) {
  if (P.nleaf == 0) return hipSuccess;
  const dim3 g(unsigned(P.nleaf)), b(256);
  switch (P.N) {
    case 8: hipLaunchKernelGGL(indicator_kernel<8>, g, b, 0, st, U, P); break;
    case 16: hipLaunchKernelGGL(indicator_kernel<16>, g, b, 0, st, U, P); break;
    case 32: hipLaunchKernelGGL(indicator_kernel<32>, g, b, 0, st, U, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_migrate(const DevPlan& P, const double* Uold, double* Unew, hipStream_t st) {
  if (P.nleaf == 0) return hipSuccess;
  const int64_t n = P.nleaf * int64_t(P.N) * P.N * P.N;
  const dim3 g(grid_for(n, 256)), b(256);
  const bool de = P.nf == kFieldsDE;
  switch (P.N) {
    case 8:
      if (de) hipLaunchKernelGGL((migrate_kernel<8, kFieldsDE>), g, b, 0, st, Uold, Unew, P);
      else hipLaunchKernelGGL((migrate_kernel<8, kFields>), g, b, 0, st, Uold, Unew, P);
      break;
    case 16:
      if (de) hipLaunchKernelGGL((migrate_kernel<16, kFieldsDE>), g, b, 0, st, Uold, Unew, P);
      else hipLaunchKernelGGL((migrate_kernel<16, kFields>), g, b, 0, st, Uold, Unew, P);
      break;
    case 32:
      if (de) hipLaunchKernelGGL((migrate_kernel<32, kFieldsDE>), g, b, 0, st, Uold, Unew, P);
      else hipLaunchKernelGGL((migrate_kernel<32, kFields>), g, b, 0, st, Uold, Unew, P);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reflux(const DevPlan& P, double* U, const double* dt, int dir, const LaunchCfg& L,
                         hipStream_t st) {
  switch (P.N) {
    case 8: return reflux_n<8>(P, U, dt, dir, L, st);
    case 16: return reflux_n<16>(P, U, dt, dir, L, st);
    case 32: return reflux_n<32>(P, U, dt, dir, L, st);
    default: return hipErrorInvalidValue;
  }
}

// Work items per leaf of the largest forward launch over the leaves: the
// staged sweep's tiles (ceil(M^2 / R) tiles of WG lanes) or one item per
// padded cell.  A dispatch counts its work items in 32 bits.
namespace {
template <int N, int DIR>
int64_t staged_items() {
  using S = StagedShape<N, DIR>;
  return int64_t((S::M * S::M + S::R - 1) / S::R) * S::WG;
}
template <int N>
int64_t forward_items() {
  constexpr int64_t M = N + 2 * G;
  return std::max({M * M * M, staged_items<N, 0>(), staged_items<N, 1>(), staged_items<N, 2>()});
}
}  // namespace

int64_t forward_items_per_leaf(int N) {
  switch (N) {
    case 8: return forward_items<8>();
    case 16: return forward_items<16>();
    default: return forward_items<32>();
  }
}

}  // namespace amr
