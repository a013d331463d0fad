// tracers.hpp -- device view of a tracer-particle set and the launchers of
// the tracer kernels (tracers.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace amr {

constexpr int kTracerBatch = 256;      // slots per batch: the unit of storage and of work
constexpr int AMR_BC_PERIODIC_DEV = 0;  // boundary code of a periodic axis in InstParams

enum TracerFlag { TRACER_OVERFLOW = 0, TRACER_REMOVED = 1, TRACER_LOST = 2, TRACER_NFLAGS = 4 };

struct TracerDev {
  double* pos_in;           // 3 planes of nleaf * cap (X, Y, Z); updated in place by the drift
  const int64_t* id_in;
  const int32_t* count_in;
  double* pos_out;
  int64_t* id_out;
  int32_t* count_out;
  int32_t* dest;            // nleaf * cap: destination leaf of each slot (-1: removed)
  int32_t* stay_batch;      // nleaf * nbatch: particles of each batch that stay in their leaf
  int32_t* stay;            // nleaf (zero between advances)
  int32_t* arrive;          // nleaf (zero between advances)
  unsigned long long* flags;  // TRACER_NFLAGS cumulative counters
  int64_t cap, plane;       // slots per leaf; nleaf * cap of the input set
  int64_t plane_out;        // nleaf * cap of the output set (differs after a remesh)
  int32_t nbatch;           // cap / kTracerBatch
};

// scratch layout (bytes, 256-aligned sections) for nleaf leaves of cap slots
struct TracerScratch {
  int64_t dest, stay_batch, stay, arrive, flags, total;
};
inline TracerScratch tracer_scratch_layout(int64_t nleaf, int64_t cap) {
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  TracerScratch L;
  int64_t o = 0;
  L.dest = o; o += up(nleaf * cap * 4);
  L.stay_batch = o; o += up(nleaf * (cap / kTracerBatch) * 4);
  L.stay = o; o += up(nleaf * 4);
  L.arrive = o; o += up(nleaf * 4);
  L.flags = o; o += up(TRACER_NFLAGS * 8);
  L.total = o;
  return L;
}

// drift + migration of every particle of T.in into T.out (U: refreshed
// state at the start of the step, dt per instance on the device)
hipError_t launch_tracers_advance(const DevPlan& P, const double* U, const double* dt, const TracerDev& T,
                                  hipStream_t st);
hipError_t launch_tracer_zero_flags(const TracerDev& T, hipStream_t st);
// move every particle of T.in (sets of the mesh before a remesh, old_nleaf
// leaves) to its leaf of the remeshed mesh P (its relocation table) in T.out
hipError_t launch_tracers_relocate(const DevPlan& P, int64_t old_nleaf, const TracerDev& T, hipStream_t st);

}  // namespace amr
