// layout.hpp -- device-visible tables of an execution plan (one or more
// meshes flattened into one worklist of leaf blocks).
//
// Every table lives in one caller-owned device workspace; offsets are
// 256-byte aligned.  The host builds the same bytes in one staging buffer and
// uploads them with a single copy.
#pragma once
#include <cstdint>

namespace amr {

constexpr int kGhost = 3;
constexpr int kFields = 5;    // rho, m_x, m_y, m_z, E
constexpr int kFieldsDE = 6;  // with the dual-energy field rho e
// slots per leaf of the next-step signal-speed maxima of a run of steps (spread
// so that a leaf's waves do not all update one word)
constexpr int kCflSlots = 16;
// Phase-2 refresh: groups of ghost cells sharing one coarse parent in a ghost
// region of kind K (0: face, 1: edge, 2: corner) of an N^3 block, and the
// whole waves a region's task takes
constexpr int p2_groups(int N, int K) { return K == 0 ? 2 * (N / 2) * (N / 2) : (K == 1 ? 4 * (N / 2) : 8); }
constexpr int p2_waves(int N, int K) { return (p2_groups(N, K) + 63) / 64; }
constexpr int kP2SubBits = 3;  // wave-in-task bits of a phase-2 wave entry (at most 8 waves per task)
// leaves from which the phase-1 refresh takes the XCD-contiguous workgroup
// order and writes the ghost cells with non-temporal stores (measured on
// gfx950, 64,567 leaves of 32^3: order 45.0 -> 40.6 ms, stores 40.7 -> 37.0
// ms; 624 leaves: 0.380 -> 0.425 and 0.374 -> 0.394 ms)
constexpr int64_t kP1LargeMinLeaves = 4096;

// Per mesh instance: gas constants in the exact forms the formulas use
// (computed once on the host in FP64) and the geometry.
struct InstParams {
  double gamma, gm1, inv_gm1, g_gm1, g1;
  double rho_floor, p_floor, cfl;
  double sixth, two3;
  double eta1, eta2;  // dual-energy thresholds (pressure selection, resynchronisation)
  int32_t root[3];
  int32_t bc[3];
  int32_t iters;
  int32_t de;  // the plan carries the dual-energy field
  int64_t first_leaf;  // first block of this instance in the plan
  int64_t n_leaf;
};
static_assert(sizeof(InstParams) % 8 == 0, "InstParams packing");

struct BlockInfo {
  int32_t level, i, j, k;
  int32_t inst;
  int32_t rflx;  // bit 2 d + side: the reflux corrects this leaf's face (d, side)
  int32_t pad[2];
};

// Neighbour of a leaf in one of the 26 directions (code = (sx+1) +
// 3 (sy+1) + 9 (sz+1), code 13 unused): where its ghost box comes from.
enum NbrKind : int32_t {
  NBR_COPY = 0,    // same-level leaf `id` (after periodic wrap or outflow clamp)
  NBR_FINE = 1,    // refined same-level position: children in fine table row `id`
  NBR_COARSE = 2,  // absent same-level position: covering leaf `id` one level up
};
struct Nbr {
  int32_t kind, id;
};

// Reflux task: a coarse leaf's face whose same-level neighbour position is
// refined.  The fine face fluxes of the 4 children touching it correct the
// coarse face cells.
struct RefluxTask {
  int32_t leaf, side, slot_c;
  int32_t slot_f[4];  // child face slots by quadrant (hA + 2 hB)
  int32_t pad;
};

// Data migration after a remesh, one task per new leaf: copy the old leaf
// `src[0]`, prolong from the old parent `src[0]` (child octant `co`), or
// restrict the 8 old children src[0..7] (x fastest, then y, then z).
enum MigrKind : int32_t { MIGR_COPY = 0, MIGR_PROLONG = 1, MIGR_RESTRICT = 2 };
struct MigrTask {
  int32_t kind, co;
  int32_t src[8];
};

// Where the particles of an old leaf go in a remeshed mesh.
enum RelocKind : int32_t { RELOC_KEEP = 0, RELOC_SPLIT = 1, RELOC_MERGE = 2 };
struct Reloc {
  int32_t kind;  // RELOC_*
  int32_t id;    // KEEP/MERGE: new leaf; SPLIT: row of 8 children (x fastest) in reloc_child
};

struct PlanOffsets {
  int64_t inst, blocks, nbr, fine, p2list, p2task, p2wave, faceslot, reflux[3], acc, lacc, dte, counters, ind, migr, reloc,
      reloc_child, faces, total;
};

}  // namespace amr
