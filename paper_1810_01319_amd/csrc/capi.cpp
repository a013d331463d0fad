// capi.cpp -- extern "C" entry points declared in include/amr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <string>

#include "../../include/amr.h"
#include "adjoint.hpp"
#include "composite.hpp"
#include "kernels.hpp"
#include "mesh.hpp"
#include "poisson.hpp"
#include "tracers.hpp"

using namespace amr;

// Event pairs around kernel phases, recorded while profiling is on.
struct Profiler {
  bool on = false;
  struct Rec {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void release_all() {
    for (auto& r : recs) {
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
  ~Profiler() {
    release_all();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// mg0 on the octree: the hierarchy of coarsened meshes of a refined mesh and
// the layout of the solver's workspace (tables of the coarser stages, per
// stage the padded correction x, right-hand side b and operator values L,
// the transfer tasks between neighbouring stages, the uniform solver's
// levels of the root grid, reduction scratch).
struct CompositeMg {
  int lmax = 0;
  std::vector<std::unique_ptr<Octree>> trees;  // stages 0 .. lmax-1 (stage lmax is the mesh)
  std::vector<Plan> plans;                     // stages 0 .. lmax-1
  std::vector<std::vector<MigrTask>> rtask;    // stage l < lmax: per leaf, from stage l+1
  std::vector<std::vector<MigrTask>> ptask;    // stage l >= 1: per leaf, from stage l-1
  std::vector<int64_t> nleaf;                  // stages 0 .. lmax
  std::vector<int64_t> off_plan, off_x, off_b, off_L, off_r, off_p;
  int64_t off_mg = 0, off_parts = 0, off_scal = 0, total = 0, tables = 0;
  double volume = 0.0;                         // volume-weighted cell count of the mesh
  std::vector<unsigned char> staging;          // bytes [0, tables) of the workspace
};

struct amr_mesh {
  std::vector<std::unique_ptr<Octree>> trees;  // one per instance
  Octree* tree = nullptr;                      // trees[0]
  Plan plan;
  unsigned char* ws = nullptr;  // caller-owned device workspace
  LaunchCfg cfg;
  Profiler prof;
  std::unique_ptr<CompositeMg> comp;  // built on first use by the Poisson entries on a refined mesh
};

namespace {

thread_local std::string g_err;

amr_status fail(amr_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

amr_status hip_fail(hipError_t e, const char* where) {
  return fail(AMR_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

amr_status to_desc(const amr_mesh_desc* d, MeshDesc& m) {
  if (!d) return fail(AMR_E_INVALID, "null descriptor");
  if (d->ghost != 3) return fail(AMR_E_INVALID, "ghost width must be 3");
  if (d->block_cells != 8 && d->block_cells != 16 && d->block_cells != 32)
    return fail(AMR_E_INVALID, "block_cells must be 8, 16 or 32");
  if (d->max_level < 0 || d->max_level > 7) return fail(AMR_E_INVALID, "max_level must be in 0..7");
  for (int a = 0; a < 3; a++) {
    if (d->root[a] < 1 || (int64_t(d->root[a]) << d->max_level) * d->block_cells >= (int64_t(1) << 30))
      return fail(AMR_E_INVALID, "root extent out of range");
    if (d->bc[a] != AMR_BC_PERIODIC && d->bc[a] != AMR_BC_OUTFLOW) return fail(AMR_E_INVALID, "bad boundary code");
  }
  if (!(d->gamma > 1.0)) return fail(AMR_E_INVALID, "gamma must exceed 1");
  if (!(d->cfl > 0.0)) return fail(AMR_E_INVALID, "cfl must be positive");
  if (!(d->rho_floor >= 1e-100) || !(d->p_floor >= 1e-100))
    return fail(AMR_E_INVALID, "density and pressure floors must be at least 1e-100");
  if (d->riemann_iters < 0 || d->riemann_iters > 64) return fail(AMR_E_INVALID, "riemann_iters out of range");
  if (d->n_refine < 0 || (d->n_refine > 0 && !d->refine)) return fail(AMR_E_INVALID, "bad refine list");
  for (int a = 0; a < 3; a++) m.root[a] = d->root[a], m.bc[a] = d->bc[a];
  m.N = d->block_cells;
  m.max_level = d->max_level;
  m.gamma = d->gamma;
  m.cfl = d->cfl;
  m.rho_floor = d->rho_floor;
  m.p_floor = d->p_floor;
  m.iters = d->riemann_iters;
  if (d->dual_energy != 0 && d->dual_energy != 1) return fail(AMR_E_INVALID, "dual_energy must be 0 or 1");
  if (d->dual_energy && !(d->eta1 >= 0.0 && d->eta1 <= 1.0 && d->eta2 >= 0.0 && d->eta2 <= 1.0))
    return fail(AMR_E_INVALID, "eta1 and eta2 must lie in [0, 1]");
  m.de = d->dual_energy;
  m.eta1 = d->dual_energy ? d->eta1 : 0.0;
  m.eta2 = d->dual_energy ? d->eta2 : 0.0;
  return AMR_OK;
}

// Leaves of N^3 that one launch over a plan's leaves can cover: a dispatch
// counts its work items in 32 bits, and the largest launches (the staged
// sweeps, their transposes, the cell-wise kernels) take a fixed number per
// leaf.
int64_t launch_leaf_limit(int N) {
  const int64_t per = std::max(forward_items_per_leaf(N), adjoint_items_per_leaf(N));
  return ((int64_t(1) << 32) - 1) / per;
}

amr_status finish(amr_mesh* h, amr_mesh** out) {
  std::vector<const Octree*> v;
  for (auto& t : h->trees) v.push_back(t.get());
  h->tree = h->trees[0].get();
  std::string e = h->plan.build(v);
  if (!e.empty()) {
    delete h;
    return fail(AMR_E_BALANCE, e);
  }
  if (h->plan.nleaf > launch_leaf_limit(h->plan.N)) {
    const std::string m = std::to_string(h->plan.nleaf) + " leaves of " + std::to_string(h->plan.N) +
                          "^3: a launch over them would exceed 2^32 work items (at most " +
                          std::to_string(launch_leaf_limit(h->plan.N)) + ")";
    delete h;
    return fail(AMR_E_INVALID, m);
  }
  for (size_t m = 0; m < h->trees.size(); m++) {
    bool outflow = false;
    for (int a = 0; a < 3; a++) outflow = outflow || h->trees[m]->desc().bc[a] == AMR_BC_OUTFLOW;
    if (!outflow) continue;
    const InstParams& ip = h->plan.inst[m];
    for (int64_t s = ip.first_leaf; s < ip.first_leaf + ip.n_leaf; s++)
      if (h->plan.keys[size_t(s)].l != 0) {
        delete h;
        return fail(AMR_E_INVALID, "outflow boundaries need a single-level mesh");
      }
  }
  *out = h;
  return AMR_OK;
}

// Adjoint scratch: face-flux adjoints (256-B rounded), then for the
// recomputing entry three states and one counter slot.
int64_t adjoint_face_bytes(const Plan& p) {
  const int64_t faces = p.nslots * p.nf * int64_t(p.N) * p.N * 8;
  return (faces + 255) / 256 * 256;
}

int64_t adjoint_scratch(const Plan& p) {
  const int64_t field = p.nleaf * p.nf * int64_t(p.M) * p.M * p.M * 8;
  return adjoint_face_bytes(p) + 3 * field + 256;
}

DevPlan dev_plan_at(const Plan& p, unsigned char* w) {
  DevPlan P{};
  P.inst = reinterpret_cast<const InstParams*>(w + p.off.inst);
  P.blocks = reinterpret_cast<const BlockInfo*>(w + p.off.blocks);
  P.nbr = reinterpret_cast<const Nbr*>(w + p.off.nbr);
  P.fine = reinterpret_cast<const int32_t*>(w + p.off.fine);
  P.p2list = reinterpret_cast<const int32_t*>(w + p.off.p2list);
  P.p2task = reinterpret_cast<const int32_t*>(w + p.off.p2task);
  P.p2wave = reinterpret_cast<const int32_t*>(w + p.off.p2wave);
  P.np2w = int64_t(p.p2wave.size());
  P.p1_large = p.nleaf >= kP1LargeMinLeaves ? 1 : 0;
  P.faceslot = reinterpret_cast<const int32_t*>(w + p.off.faceslot);
  for (int d = 0; d < 3; d++) {
    P.reflux[d] = reinterpret_cast<const RefluxTask*>(w + p.off.reflux[d]);
    P.nreflux[d] = int64_t(p.reflux[d].size());
  }
  P.acc = reinterpret_cast<unsigned long long*>(w + p.off.acc);
  P.lacc = reinterpret_cast<unsigned long long*>(w + p.off.lacc);
  P.dte = reinterpret_cast<double*>(w + p.off.dte);
  P.counters = reinterpret_cast<unsigned long long*>(w + p.off.counters);
  P.ind = reinterpret_cast<double*>(w + p.off.ind);
  P.migr = reinterpret_cast<const MigrTask*>(w + p.off.migr);
  P.reloc = reinterpret_cast<const Reloc*>(w + p.off.reloc);
  P.reloc_child = reinterpret_cast<const int32_t*>(w + p.off.reloc_child);
  P.faces = reinterpret_cast<double*>(w + p.off.faces);
  P.nleaf = p.nleaf;
  P.np2 = int64_t(p.p2list.size());
  for (int k = 0; k < 3; k++) P.np2t[k] = p.np2t[k];
  P.ninst = int32_t(p.inst.size());
  P.N = p.N;
  P.nf = p.nf;
  return P;
}

DevPlan dev_plan(const amr_mesh* h) { return dev_plan_at(h->plan, h->ws); }

amr_status check_ready(const amr_mesh* h, const void* U) {
  if (!h) return fail(AMR_E_INVALID, "null mesh");
  if (!h->ws) return fail(AMR_E_STATE, "no workspace uploaded (call amr_mesh_upload first)");
  if (!U) return fail(AMR_E_INVALID, "null field pointer");
  return AMR_OK;
}

// Runs `launch` between two recorded events when profiling is on.
template <class F>
hipError_t timed(amr_mesh* h, int phase, hipStream_t st, F&& launch) {
  if (!h->prof.on) return launch();
  hipEvent_t a = h->prof.get(), b = h->prof.get();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  h->prof.recs.push_back({phase, a, b});
  return e;
}

hipError_t refresh_timed(amr_mesh* h, const DevPlan& P, double* U, hipStream_t st) {
  LaunchCfg c = h->cfg;
  DevPlan p1 = P;
  p1.np2 = 0;  // phase 1 only
  hipError_t e = timed(h, AMR_PHASE_REFRESH1, st, [&] { return launch_refresh(p1, U, c, st); });
  if (e != hipSuccess || P.np2 == 0) return e;
  DevPlan p2 = P;
  p2.nleaf = 0;  // phase 2 only
  return timed(h, AMR_PHASE_REFRESH2, st, [&] { return launch_refresh(p2, U, c, st); });
}

// One step: refresh U in place, then sweep k reads the previous result and
// writes out[k] (all equal to U for the in-place step), then reflux out[2].
// cfl_next (in place only): the step also accumulates the next step's CFL
// candidates (last sweep, then the refluxed cells) into the instance
// accumulators, for cfl_finalize.
amr_status run_step_into(amr_mesh* h, double* U, double* const out[3], const double* dt, int64_t step_index,
                         hipStream_t st, const TracerDev* tracers = nullptr, int cfl_next = 0,
                         bool ghosts_fresh = false) {
  const DevPlan P = dev_plan(h);
  hipError_t e = ghosts_fresh ? hipSuccess : refresh_timed(h, P, U, st);
  if (e != hipSuccess) return hip_fail(e, "refresh");
  if (tracers) {  // drift with the refreshed start-of-step state, then migrate
    e = timed(h, AMR_PHASE_TRACERS, st, [&] { return launch_tracers_advance(P, U, dt, *tracers, st); });
    if (e != hipSuccess) return hip_fail(e, "tracers");
  }
  int order[3] = {0, 1, 2};
  if (step_index & 1) {
    order[0] = 2;
    order[2] = 0;
  }
  int swept[3] = {0, 0, 0};
  const double* in = U;
  for (int s = 0; s < 3; s++) {
    const int last = s == 2 ? cfl_next : 0;
    e = timed(h, AMR_PHASE_SWEEP_X + order[s], st,
              [&] { return launch_sweep_oop(P, in, out[s], dt, order[s], swept, h->cfg, st, last); });
    if (e != hipSuccess) return hip_fail(e, "sweep");
    swept[order[s]] = 1;
    in = out[s];
  }
  for (int d = 0; d < 3; d++) {
    if (P.nreflux[d] == 0) continue;
    e = timed(h, AMR_PHASE_REFLUX, st, [&] { return launch_reflux(P, out[2], dt, d, h->cfg, st); });
    if (e != hipSuccess) return hip_fail(e, "reflux");
  }
  if (cfl_next) {
    e = timed(h, AMR_PHASE_CFL, st, [&] { return launch_reflux_cfl(P, out[2], st); });
    if (e != hipSuccess) return hip_fail(e, "cfl");
  }
  return AMR_OK;
}

amr_status run_step(amr_mesh* h, double* U, const double* dt, int64_t step_index, hipStream_t st) {
  double* const out[3] = {U, U, U};
  return run_step_into(h, U, out, dt, step_index, st);
}

// The transposes of one step in reverse order, given the inputs S[k] of its
// three sweeps (S[0] the refreshed input state).
hipError_t adjoint_transposes(amr_mesh* h, const DevPlan& P, const double* const S[3], const double* dt,
                              const unsigned long long* floors, int64_t floors_host, double* lam, double* gfaces,
                              int64_t step_index, hipStream_t st) {
  const Plan& p = h->plan;
  int order[3] = {0, 1, 2};
  if (step_index & 1) {
    order[0] = 2;
    order[2] = 0;
  }
  hipError_t e = timed(h, AMR_PHASE_ADJ_REFLUX, st, [&] {
    hipError_t r = launch_fill_zero(gfaces, p.nslots * p.nf * int64_t(p.N) * p.N, st);
    if (r == hipSuccess) r = launch_reflux_adjoint(P, lam, dt, gfaces, st);
    return r;
  });
  for (int k = 2; k >= 0 && e == hipSuccess; k--) {
    int sw[3] = {0, 0, 0};
    for (int q = 0; q < k; q++) sw[order[q]] = 1;
    e = timed(h, AMR_PHASE_ADJ_SWEEP_X + order[k], st,
              [&] { return launch_sweep_adjoint(P, S[k], lam, dt, gfaces, floors, floors_host, order[k], sw, st); });
  }
  if (e == hipSuccess)
    e = timed(h, AMR_PHASE_ADJ_REFRESH, st, [&] { return launch_refresh_adjoint(P, lam, S[0], st); });
  return e;
}

bool adjoint_iters_ok(const Plan& p) {
  for (const InstParams& ip : p.inst)
    if (ip.iters > kAdjMaxIters) return false;
  return true;
}

amr_status decide(amr_mesh* h, const std::vector<double>& S, const amr_remesh_params* prm, amr_mesh** out,
                  amr_remesh_stats* stats) {
  // refinements beyond what one launch can cover are refused like those beyond max_blocks
  const int64_t cap = std::min<int64_t>(prm->max_blocks, launch_leaf_limit(h->plan.N));
  RemeshResult r = remesh_decide(*h->tree, h->plan, S, prm->refine_slope, prm->coarsen_slope, cap);
  if (r.refined == 0 && r.coarsened == 0) {  // the same leaves in the same order: no new mesh
    *out = nullptr;
    stats->refined = 0;
    stats->coarsened = 0;
    stats->refused = r.refused;
    stats->n_leaves = h->plan.nleaf;
    return AMR_OK;
  }
  amr_mesh* nh = new (std::nothrow) amr_mesh();
  if (!nh) return fail(AMR_E_NOMEM, "out of host memory");
  nh->trees.push_back(std::move(r.tree));
  // where the particles of each old leaf go: the inverse of the migration tasks
  std::vector<Reloc> reloc(size_t(h->plan.nleaf), Reloc{-1, -1});
  std::vector<int32_t> child;
  std::vector<int32_t> row(size_t(h->plan.nleaf), -1);
  for (size_t n = 0; n < r.migr.size(); n++) {
    const MigrTask& t = r.migr[n];
    if (t.kind == MIGR_COPY) {
      reloc[size_t(t.src[0])] = Reloc{RELOC_KEEP, int32_t(n)};
    } else if (t.kind == MIGR_PROLONG) {
      int32_t& rw = row[size_t(t.src[0])];
      if (rw < 0) {
        rw = int32_t(child.size() / 8);
        child.resize(child.size() + 8, -1);
      }
      reloc[size_t(t.src[0])] = Reloc{RELOC_SPLIT, rw};
      child[size_t(8 * rw + t.co)] = int32_t(n);
    } else {
      for (int q = 0; q < 8; q++) reloc[size_t(t.src[q])] = Reloc{RELOC_MERGE, int32_t(n)};
    }
  }
  for (const Reloc& x : reloc)
    if (x.kind < 0) {
      delete nh;
      return fail(AMR_E_STATE, "remesh left an old leaf without a successor");
    }
  for (int32_t c : child)
    if (c < 0) {
      delete nh;
      return fail(AMR_E_STATE, "remesh split a leaf into fewer than 8 children");
    }
  nh->plan.reloc = std::move(reloc);
  nh->plan.reloc_child = std::move(child);
  nh->plan.migr = std::move(r.migr);
  nh->cfg = h->cfg;
  amr_status rc = finish(nh, out);
  if (rc != AMR_OK) return rc;
  stats->refined = r.refined;
  stats->coarsened = r.coarsened;
  stats->refused = r.refused;
  stats->n_leaves = (*out)->plan.nleaf;
  return AMR_OK;
}

}  // namespace

extern "C" {

amr_status amr_mesh_create(const amr_mesh_desc* desc, amr_mesh** out) {
  if (!out) return fail(AMR_E_INVALID, "null output pointer");
  *out = nullptr;
  MeshDesc m{};
  amr_status rc = to_desc(desc, m);
  if (rc != AMR_OK) return rc;
  amr_mesh* h = new (std::nothrow) amr_mesh();
  if (!h) return fail(AMR_E_NOMEM, "out of host memory");
  h->trees.emplace_back(new Octree(m));
  std::string e = h->trees[0]->refine_list(desc->refine, desc->n_refine);
  if (!e.empty()) {
    delete h;
    return fail(AMR_E_INVALID, e);
  }
  return finish(h, out);
}

amr_status amr_mesh_create_from_leaves(const amr_mesh_desc* desc, int64_t n, const int32_t* keys,
                                       amr_mesh** out) {
  if (!out) return fail(AMR_E_INVALID, "null output pointer");
  *out = nullptr;
  MeshDesc m{};
  amr_status rc = to_desc(desc, m);
  if (rc != AMR_OK) return rc;
  if (n <= 0 || !keys) return fail(AMR_E_INVALID, "empty leaf list");
  amr_mesh* h = new (std::nothrow) amr_mesh();
  if (!h) return fail(AMR_E_NOMEM, "out of host memory");
  h->trees.emplace_back(new Octree(m));
  std::string e = h->trees[0]->from_leaves(keys, n);
  if (!e.empty()) {
    delete h;
    return fail(AMR_E_BALANCE, e);
  }
  return finish(h, out);
}

amr_status amr_batch_create(const amr_mesh_desc* descs, int32_t n, amr_batch** out) {
  if (!out || !descs || n < 1) return fail(AMR_E_INVALID, "need at least one descriptor");
  *out = nullptr;
  amr_mesh* h = new (std::nothrow) amr_mesh();
  if (!h) return fail(AMR_E_NOMEM, "out of host memory");
  for (int32_t i = 0; i < n; i++) {
    MeshDesc m{};
    amr_status rc = to_desc(&descs[i], m);
    if (rc != AMR_OK) {
      delete h;
      return rc;
    }
    if (m.N != descs[0].block_cells) {
      delete h;
      return fail(AMR_E_INVALID, "all instances of a batch need the same block_cells");
    }
    h->trees.emplace_back(new Octree(m));
    std::string e = h->trees.back()->refine_list(descs[i].refine, descs[i].n_refine);
    if (!e.empty()) {
      delete h;
      return fail(AMR_E_INVALID, "instance " + std::to_string(i) + ": " + e);
    }
  }
  return finish(h, out);
}

amr_status amr_mesh_instance_offsets(const amr_mesh* h, int64_t* first_leaf, int64_t cap) {
  if (!h || !first_leaf) return fail(AMR_E_INVALID, "null argument");
  const int64_t n = int64_t(h->plan.inst.size());
  if (cap < n + 1) return fail(AMR_E_INVALID, "output too small");
  for (int64_t m = 0; m < n; m++) first_leaf[m] = h->plan.inst[size_t(m)].first_leaf;
  first_leaf[n] = h->plan.nleaf;
  return AMR_OK;
}

amr_status amr_mesh_destroy(amr_mesh* mesh) {
  delete mesh;
  return AMR_OK;
}

amr_status amr_mesh_info(const amr_mesh* h, amr_mesh_info_t* out) {
  if (!h || !out) return fail(AMR_E_INVALID, "null argument");
  std::memset(out, 0, sizeof *out);
  const Plan& p = h->plan;
  out->n_leaves = p.nleaf;
  out->block_cells = p.N;
  out->padded = p.M;
  out->field_stride = int64_t(p.M) * p.M * p.M;
  out->block_stride = p.nf * out->field_stride;
  out->n_fields = p.nf;
  out->field_bytes = p.nleaf * out->block_stride * 8;
  out->workspace_bytes = p.off.total;
  out->n_cf_faces = p.nslots;
  out->n_instances = int64_t(p.inst.size());
  out->adjoint_scratch_bytes = adjoint_scratch(p);
  out->adjoint_face_bytes = adjoint_face_bytes(p);
  for (const Key& k : p.keys)
    if (k.l < 8) out->levels[k.l]++;
  return AMR_OK;
}

amr_status amr_mesh_blocks(const amr_mesh* h, int32_t* keys_out, int64_t cap) {
  if (!h || !keys_out) return fail(AMR_E_INVALID, "null argument");
  if (cap < h->plan.nleaf) return fail(AMR_E_INVALID, "output too small");
  for (int64_t s = 0; s < h->plan.nleaf; s++) {
    const Key& k = h->plan.keys[size_t(s)];
    keys_out[4 * s] = k.l;
    keys_out[4 * s + 1] = k.i;
    keys_out[4 * s + 2] = k.j;
    keys_out[4 * s + 3] = k.k;
  }
  return AMR_OK;
}

amr_status amr_mesh_upload(amr_mesh* h, void* ws, void* stream) {
  if (!h || !ws) return fail(AMR_E_INVALID, "null argument");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(AMR_E_INVALID, "workspace must be 256-byte aligned");
  hipError_t e = hipMemcpyAsync(ws, h->plan.staging.data(), h->plan.staging.size(), hipMemcpyHostToDevice,
                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "upload");
  h->ws = static_cast<unsigned char*>(ws);
  return AMR_OK;
}

amr_status amr_refresh_ghosts(amr_mesh* h, double* U, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  hipError_t e = refresh_timed(h, dev_plan(h), U, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? AMR_OK : hip_fail(e, "refresh");
}

amr_status amr_cfl_dt(amr_mesh* h, const double* U, double* dt, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt) return fail(AMR_E_INVALID, "null dt pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  hipError_t e = timed(h, AMR_PHASE_CFL, st, [&] { return launch_cfl(P, U, dt, h->cfg, st); });
  return e == hipSuccess ? AMR_OK : hip_fail(e, "cfl");
}

amr_status amr_hydro_step(amr_mesh* h, double* U, double* dt, int64_t step_index, void* stream) {
  amr_status rc = amr_cfl_dt(h, U, dt, stream);
  if (rc != AMR_OK) return rc;
  return run_step(h, U, dt, step_index, static_cast<hipStream_t>(stream));
}

amr_status amr_batch_step(amr_batch* b, double* U, double* dt, int64_t step_index, void* stream) {
  return amr_hydro_step(b, U, dt, step_index, stream);
}

namespace {
amr_status hydro_steps(amr_mesh* h, double* U, double* dt, int64_t nsteps, int64_t first_step, void* stream,
                       bool ghosts_fresh) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt) return fail(AMR_E_INVALID, "null dt pointer");
  if (nsteps < 0) return fail(AMR_E_INVALID, "negative step count");
  if (nsteps == 0) return AMR_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  hipError_t e = timed(h, AMR_PHASE_CFL, st, [&] { return launch_cfl(P, U, dt, h->cfg, st); });
  if (e != hipSuccess) return hip_fail(e, "cfl");
  double* const out[3] = {U, U, U};
  for (int64_t i = 0; i < nsteps; i++) {
    double* const dti = dt + i * P.ninst;
    if (i > 0) {
      e = timed(h, AMR_PHASE_CFL, st, [&] { return launch_cfl_finalize(P, dti, st); });
      if (e != hipSuccess) return hip_fail(e, "cfl");
    }
    rc = run_step_into(h, U, out, dti, first_step + i, st, nullptr, i + 1 < nsteps ? 1 : 0, ghosts_fresh && i == 0);
    if (rc != AMR_OK) return rc;
  }
  return AMR_OK;
}
}  // namespace

amr_status amr_hydro_steps(amr_mesh* h, double* U, double* dt, int64_t nsteps, int64_t first_step, void* stream) {
  return hydro_steps(h, U, dt, nsteps, first_step, stream, false);
}

amr_status amr_hydro_steps_fresh(amr_mesh* h, double* U, double* dt, int64_t nsteps, int64_t first_step,
                                 void* stream) {
  return hydro_steps(h, U, dt, nsteps, first_step, stream, true);
}

amr_status amr_hydro_step_dt(amr_mesh* h, double* U, const double* dt, int64_t step_index, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt) return fail(AMR_E_INVALID, "null dt pointer");
  return run_step(h, U, dt, step_index, static_cast<hipStream_t>(stream));
}

amr_status amr_cfl_dt_comoving(amr_mesh* h, const double* U, double a, double* dt, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt) return fail(AMR_E_INVALID, "null dt pointer");
  if (!(a > 0.0) || !std::isfinite(a)) return fail(AMR_E_INVALID, "expansion factor must be positive and finite");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  hipError_t e = timed(h, AMR_PHASE_CFL, st, [&] { return launch_cfl(P, U, dt, h->cfg, st, a); });
  return e == hipSuccess ? AMR_OK : hip_fail(e, "cfl");
}

amr_status amr_hydro_step_comoving(amr_mesh* h, double* U, const double* dt, int64_t step_index, double a,
                                   double hubble, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt) return fail(AMR_E_INVALID, "null dt pointer");
  if (!(a > 0.0) || !std::isfinite(a)) return fail(AMR_E_INVALID, "expansion factor must be positive and finite");
  if (!std::isfinite(hubble)) return fail(AMR_E_INVALID, "expansion rate must be finite");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  hipError_t e = launch_scale_dt(P, dt, a, st);
  if (e != hipSuccess) return hip_fail(e, "comoving dt");
  rc = run_step(h, U, P.dte, step_index, st);
  if (rc != AMR_OK) return rc;
  e = timed(h, AMR_PHASE_EXPANSION, st, [&] { return launch_expansion(P, U, dt, hubble, st); });
  return e == hipSuccess ? AMR_OK : hip_fail(e, "expansion");
}

amr_status amr_hydro_steps_comoving(amr_mesh* h, double* U, double* dt, int64_t nsteps, int64_t first_step,
                                    double H0, double omega_m, double omega_l, double* cosmo, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt || !cosmo) return fail(AMR_E_INVALID, "null argument");
  if (nsteps < 0) return fail(AMR_E_INVALID, "nsteps < 0");
  if (h->plan.inst.size() != 1) return fail(AMR_E_INVALID, "a run of comoving steps needs a single mesh");
  if (!(H0 > 0.0) || !std::isfinite(H0) || !(omega_m > 0.0) || !(omega_l >= 0.0) ||
      !(std::fabs(omega_m + omega_l - 1.0) <= 1e-12))
    return fail(AMR_E_INVALID, "cosmology: H0 > 0, omega_m > 0, omega_l >= 0, omega_m + omega_l = 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  for (int64_t k = 0; k < nsteps; k++) {
    double* const dk = dt + k;
    hipError_t e = launch_cosmology(0, H0, omega_m, omega_l, dk, cosmo, st);
    if (e == hipSuccess)
      e = timed(h, AMR_PHASE_CFL, st, [&] { return launch_cfl(P, U, dk, h->cfg, st, 1.0, cosmo + 1); });
    if (e == hipSuccess) e = launch_cosmology(1, H0, omega_m, omega_l, dk, cosmo, st);
    if (e == hipSuccess) e = launch_scale_dt(P, dk, 1.0, st, cosmo + 2);
    if (e != hipSuccess) return hip_fail(e, "comoving dt");
    rc = run_step(h, U, P.dte, first_step + k, st);
    if (rc != AMR_OK) return rc;
    e = timed(h, AMR_PHASE_EXPANSION, st, [&] { return launch_expansion(P, U, dk, 0.0, st, cosmo + 3); });
    if (e != hipSuccess) return hip_fail(e, "expansion");
  }
  return AMR_OK;
}

amr_status amr_hydro_step_record(amr_mesh* h, double* U, double* dt, double* S1, double* S2, double* Uout,
                                 uint64_t* floors, int64_t step_index, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt || !S1 || !S2 || !Uout || !floors) return fail(AMR_E_INVALID, "null argument");
  if (S1 == U || S2 == U || Uout == U || S1 == S2 || S1 == Uout || S2 == Uout)
    return fail(AMR_E_INVALID, "U, S1, S2 and U_out must be distinct buffers");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  unsigned long long* mark = reinterpret_cast<unsigned long long*>(floors);
  hipError_t e = launch_floor_mark(P, mark, 0, st);
  if (e != hipSuccess) return hip_fail(e, "floor mark");
  rc = amr_cfl_dt(h, U, dt, stream);
  if (rc != AMR_OK) return rc;
  double* const out[3] = {S1, S2, Uout};
  rc = run_step_into(h, U, out, dt, step_index, st);
  if (rc != AMR_OK) return rc;
  e = launch_floor_mark(P, mark, 1, st);
  return e == hipSuccess ? AMR_OK : hip_fail(e, "floor mark");
}

amr_status amr_hydro_step_adjoint(amr_mesh* h, const double* Uin, const double* dt, double* lam, void* scratch,
                                  int64_t step_index, void* stream) {
  amr_status rc = check_ready(h, Uin);
  if (rc != AMR_OK) return rc;
  if (!dt || !lam || !scratch) return fail(AMR_E_INVALID, "null argument");
  const Plan& p = h->plan;
  if (!adjoint_iters_ok(p)) return fail(AMR_E_INVALID, "adjoint supports riemann_iters <= 8");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nfield = p.nleaf * p.nf * int64_t(p.M) * p.M * p.M;
  unsigned char* sc = static_cast<unsigned char*>(scratch);
  double* gfaces = reinterpret_cast<double*>(sc);
  double* S[3];
  for (int i = 0; i < 3; i++) S[i] = reinterpret_cast<double*>(sc + adjoint_face_bytes(p)) + i * nfield;
  unsigned long long* mark = reinterpret_cast<unsigned long long*>(S[2] + nfield);
  const DevPlan P = dev_plan(h);
  int order[3] = {0, 1, 2};
  if (step_index & 1) {
    order[0] = 2;
    order[2] = 0;
  }
  // recompute the inputs of the three sweeps; the floor-reset counter is
  // restored afterwards so that recomputation does not count twice
  int swept[3] = {0, 0, 0};
  hipError_t e = timed(h, AMR_PHASE_ADJ_RECOMPUTE, st, [&] {
    hipError_t r = launch_floor_mark(P, mark, 0, st);
    if (r == hipSuccess) r = hipMemcpyAsync(S[0], Uin, size_t(nfield) * 8, hipMemcpyDeviceToDevice, st);
    if (r == hipSuccess) r = launch_refresh(P, S[0], h->cfg, st);
    for (int k = 0; k < 2 && r == hipSuccess; k++) {
      r = launch_sweep_oop(P, S[k], S[k + 1], dt, order[k], swept, h->cfg, st);
      swept[order[k]] = 1;
    }
    if (r == hipSuccess) r = launch_floor_mark(P, mark, 2, st);
    return r;
  });
  if (e != hipSuccess) return hip_fail(e, "adjoint recompute");
  const double* const Sc[3] = {S[0], S[1], S[2]};
  e = adjoint_transposes(h, P, Sc, dt, nullptr, -1, lam, gfaces, step_index, st);
  return e == hipSuccess ? AMR_OK : hip_fail(e, "adjoint");
}

amr_status amr_hydro_step_adjoint_recorded(amr_mesh* h, const double* S0, const double* S1, const double* S2,
                                           const double* dt, const uint64_t* floors, int64_t floors_host,
                                           double* lam, void* scratch, int64_t step_index, void* stream) {
  amr_status rc = check_ready(h, S0);
  if (rc != AMR_OK) return rc;
  if (!S1 || !S2 || !dt || !lam || !scratch) return fail(AMR_E_INVALID, "null argument");
  if (floors_host < -1) return fail(AMR_E_INVALID, "floors_host must be a count or -1");
  if (!adjoint_iters_ok(h->plan)) return fail(AMR_E_INVALID, "adjoint supports riemann_iters <= 8");
  const double* const S[3] = {S0, S1, S2};
  hipError_t e = adjoint_transposes(h, dev_plan(h), S, dt, reinterpret_cast<const unsigned long long*>(floors),
                                    floors ? floors_host : -1, lam, static_cast<double*>(scratch), step_index,
                                    static_cast<hipStream_t>(stream));
  return e == hipSuccess ? AMR_OK : hip_fail(e, "adjoint");
}

amr_status amr_hydro_step_comoving_record(amr_mesh* h, double* U, const double* dt, double a, double hubble,
                                          double* S1, double* S2, double* Upre, double* Uout, uint64_t* floors,
                                          int64_t step_index, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt || !S1 || !S2 || !Upre || !Uout || !floors) return fail(AMR_E_INVALID, "null argument");
  const double* const bufs[5] = {U, S1, S2, Upre, Uout};
  for (int i = 0; i < 5; i++)
    for (int j = i + 1; j < 5; j++)
      if (bufs[i] == bufs[j]) return fail(AMR_E_INVALID, "U, S1, S2, U_pre and U_out must be distinct buffers");
  if (!(a > 0.0) || !std::isfinite(a)) return fail(AMR_E_INVALID, "expansion factor must be positive and finite");
  if (!std::isfinite(hubble)) return fail(AMR_E_INVALID, "expansion rate must be finite");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  unsigned long long* mark = reinterpret_cast<unsigned long long*>(floors);
  hipError_t e = launch_floor_mark(P, mark, 0, st);
  if (e == hipSuccess) e = launch_scale_dt(P, dt, a, st);
  if (e != hipSuccess) return hip_fail(e, "comoving record");
  double* const out[3] = {S1, S2, Upre};
  rc = run_step_into(h, U, out, P.dte, step_index, st);
  if (rc != AMR_OK) return rc;
  // the sweeps' resets only: the adjoint's floor transposes depend on them
  e = launch_floor_mark(P, mark, 1, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(Uout, Upre, size_t(h->plan.nleaf) * h->plan.nf * size_t(h->plan.M) * h->plan.M * h->plan.M *
                                       sizeof(double),
                       hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = timed(h, AMR_PHASE_EXPANSION, st, [&] { return launch_expansion(P, Uout, dt, hubble, st); });
  return e == hipSuccess ? AMR_OK : hip_fail(e, "comoving record");
}

amr_status amr_hydro_step_comoving_adjoint_recorded(amr_mesh* h, const double* S0, const double* S1,
                                                    const double* S2, const double* Upre, const double* dt, double a,
                                                    double hubble, const uint64_t* floors, int64_t floors_host,
                                                    double* lam, void* scratch, int64_t step_index, void* stream) {
  amr_status rc = check_ready(h, S0);
  if (rc != AMR_OK) return rc;
  if (!S1 || !S2 || !Upre || !dt || !lam || !scratch) return fail(AMR_E_INVALID, "null argument");
  if (floors_host < -1) return fail(AMR_E_INVALID, "floors_host must be a count or -1");
  if (!(a > 0.0) || !std::isfinite(a)) return fail(AMR_E_INVALID, "expansion factor must be positive and finite");
  if (!std::isfinite(hubble)) return fail(AMR_E_INVALID, "expansion rate must be finite");
  if (!adjoint_iters_ok(h->plan)) return fail(AMR_E_INVALID, "adjoint supports riemann_iters <= 8");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  hipError_t e = launch_expansion_adjoint(P, Upre, lam, dt, hubble, st);
  if (e == hipSuccess) e = launch_scale_dt(P, dt, a, st);
  if (e != hipSuccess) return hip_fail(e, "comoving adjoint");
  const double* const S[3] = {S0, S1, S2};
  e = adjoint_transposes(h, P, S, P.dte, reinterpret_cast<const unsigned long long*>(floors),
                         floors ? floors_host : -1, lam, static_cast<double*>(scratch), step_index, st);
  return e == hipSuccess ? AMR_OK : hip_fail(e, "comoving adjoint");
}

// ---- tracer particles ------------------------------------------------------

amr_status tracer_dev(amr_mesh* h, const amr_tracer_set_t* in, amr_tracer_set_t* out, int64_t cap, void* scratch,
                      TracerDev* T) {
  if (!in || !scratch) return fail(AMR_E_INVALID, "null argument");
  if (!in->pos || !in->id || !in->count) return fail(AMR_E_INVALID, "null input tracer array");
  if (cap <= 0 || cap % kTracerBatch != 0 || cap > (int64_t(1) << 30))
    return fail(AMR_E_INVALID, "capacity must be a positive multiple of 256");
  if (out) {
    if (!out->pos || !out->id || !out->count) return fail(AMR_E_INVALID, "null output tracer array");
    if (out->pos == in->pos || out->id == in->id || out->count == in->count)
      return fail(AMR_E_INVALID, "input and output tracer sets must be distinct");
  }
  const int64_t nleaf = h->plan.nleaf;
  // the tracer kernels run one lane per slot of every leaf in one launch
  if (nleaf * cap >= (int64_t(1) << 32))
    return fail(AMR_E_INVALID, "leaves x capacity reach 2^32 slots: more than one launch can cover");
  const TracerScratch L = tracer_scratch_layout(nleaf, cap);
  unsigned char* sc = static_cast<unsigned char*>(scratch);
  T->pos_in = in->pos;
  T->id_in = in->id;
  T->count_in = in->count;
  T->pos_out = out ? out->pos : nullptr;
  T->id_out = out ? out->id : nullptr;
  T->count_out = out ? out->count : nullptr;
  T->dest = reinterpret_cast<int32_t*>(sc + L.dest);
  T->stay_batch = reinterpret_cast<int32_t*>(sc + L.stay_batch);
  T->stay = reinterpret_cast<int32_t*>(sc + L.stay);
  T->arrive = reinterpret_cast<int32_t*>(sc + L.arrive);
  T->flags = reinterpret_cast<unsigned long long*>(sc + L.flags);
  T->cap = cap;
  T->plane = nleaf * cap;
  T->plane_out = nleaf * cap;
  T->nbatch = int32_t(cap / kTracerBatch);
  return AMR_OK;
}

amr_status amr_tracer_scratch_bytes(const amr_mesh* h, int64_t capacity, int64_t* bytes) {
  if (!h || !bytes) return fail(AMR_E_INVALID, "null argument");
  if (capacity <= 0 || capacity % kTracerBatch != 0) return fail(AMR_E_INVALID, "capacity must be a multiple of 256");
  *bytes = tracer_scratch_layout(h->plan.nleaf, capacity).total;
  return AMR_OK;
}

amr_status amr_tracers_advance(amr_mesh* h, const double* U, const double* dt, const amr_tracer_set_t* in,
                               amr_tracer_set_t* out, int64_t capacity, void* scratch, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt || !out) return fail(AMR_E_INVALID, "null argument");
  TracerDev T;
  rc = tracer_dev(h, in, out, capacity, scratch, &T);
  if (rc != AMR_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = timed(h, AMR_PHASE_TRACERS, st, [&] { return launch_tracers_advance(dev_plan(h), U, dt, T, st); });
  return e == hipSuccess ? AMR_OK : hip_fail(e, "tracers");
}

amr_status amr_hydro_step_tracers(amr_mesh* h, double* U, double* dt, const amr_tracer_set_t* in,
                                  amr_tracer_set_t* out, int64_t capacity, void* scratch, int64_t step_index,
                                  void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!out) return fail(AMR_E_INVALID, "null argument");
  TracerDev T;
  rc = tracer_dev(h, in, out, capacity, scratch, &T);
  if (rc != AMR_OK) return rc;
  rc = amr_cfl_dt(h, U, dt, stream);
  if (rc != AMR_OK) return rc;
  double* const o[3] = {U, U, U};
  return run_step_into(h, U, o, dt, step_index, static_cast<hipStream_t>(stream), &T);
}

amr_status amr_tracers_remesh(amr_mesh* nh, int64_t old_leaves, const amr_tracer_set_t* old_set,
                              amr_tracer_set_t* new_set, int64_t capacity, void* scratch, void* stream) {
  if (!nh || !new_set) return fail(AMR_E_INVALID, "null argument");
  if (!nh->ws) return fail(AMR_E_STATE, "mesh not uploaded");
  if (nh->plan.reloc.size() != size_t(old_leaves))
    return fail(AMR_E_STATE, "mesh was not made by amr_remesh_plan from a mesh of old_leaves leaves");
  TracerDev T;
  amr_status rc = tracer_dev(nh, old_set, new_set, capacity, scratch, &T);
  if (rc != AMR_OK) return rc;
  T.plane = old_leaves * capacity;  // the input set belongs to the old mesh
  hipError_t e = launch_tracers_relocate(dev_plan(nh), old_leaves, T, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? AMR_OK : hip_fail(e, "tracer relocation");
}

amr_status amr_tracer_counters(amr_mesh* h, void* scratch, int64_t capacity, int64_t* out3, int32_t reset,
                               void* stream) {
  if (!h || !scratch || !out3) return fail(AMR_E_INVALID, "null argument");
  if (capacity <= 0 || capacity % kTracerBatch != 0) return fail(AMR_E_INVALID, "capacity must be a multiple of 256");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const TracerScratch L = tracer_scratch_layout(h->plan.nleaf, capacity);
  unsigned long long f[TRACER_NFLAGS];
  hipError_t e = hipMemcpyAsync(f, static_cast<unsigned char*>(scratch) + L.flags, sizeof f, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "tracer counters");
  out3[0] = int64_t(f[TRACER_OVERFLOW]);
  out3[1] = int64_t(f[TRACER_REMOVED]);
  out3[2] = int64_t(f[TRACER_LOST]);
  if (reset) {
    TracerDev T{};
    T.flags = reinterpret_cast<unsigned long long*>(static_cast<unsigned char*>(scratch) + L.flags);
    e = launch_tracer_zero_flags(T, st);
    if (e != hipSuccess) return hip_fail(e, "tracer counters");
  }
  return AMR_OK;
}

amr_status amr_refresh_ghosts_adjoint(amr_mesh* h, const double* Uref, double* lam, void* stream) {
  amr_status rc = check_ready(h, Uref);
  if (rc != AMR_OK) return rc;
  if (!lam) return fail(AMR_E_INVALID, "null adjoint");
  hipError_t e = launch_refresh_adjoint(dev_plan(h), lam, Uref, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? AMR_OK : hip_fail(e, "refresh adjoint");
}

amr_status amr_floor_count(amr_mesh* h, int64_t* out, void* stream) {
  if (!h || !out) return fail(AMR_E_INVALID, "null argument");
  if (!h->ws) return fail(AMR_E_STATE, "no workspace uploaded");
  unsigned long long v = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&v, h->ws + h->plan.off.counters, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "floor count");
  *out = int64_t(v);
  return AMR_OK;
}

amr_status amr_indicator(amr_mesh* h, const double* U, double* ind, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!ind) return fail(AMR_E_INVALID, "null output");
  hipStream_t st = static_cast<hipStream_t>(stream);
  DevPlan P = dev_plan(h);
  P.ind = ind;
  hipError_t e = launch_indicator(P, U, st);
  return e == hipSuccess ? AMR_OK : hip_fail(e, "indicator");
}

amr_status amr_remesh_plan(amr_mesh* h, double* U, const amr_remesh_params* prm, amr_mesh** out,
                           amr_remesh_stats* stats, void* stream) {
  if (!out || !prm || !stats) return fail(AMR_E_INVALID, "null argument");
  *out = nullptr;
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (h->plan.inst.size() != 1) return fail(AMR_E_INVALID, "remesh works on single meshes");
  if (prm->max_blocks < h->plan.nleaf)
    return fail(AMR_E_CAPACITY, "max_blocks below the current leaf count");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  hipError_t e = refresh_timed(h, P, U, st);
  if (e == hipSuccess) e = launch_indicator(P, U, st);
  std::vector<double> S(size_t(h->plan.nleaf));
  if (e == hipSuccess) e = hipMemcpyAsync(S.data(), P.ind, S.size() * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "remesh indicator");
  return decide(h, S, prm, out, stats);
}

amr_status amr_remesh_plan_host(amr_mesh* h, const double* S_host, const amr_remesh_params* prm, amr_mesh** out,
                                amr_remesh_stats* stats) {
  if (!h || !S_host || !prm || !out || !stats) return fail(AMR_E_INVALID, "null argument");
  *out = nullptr;
  if (h->plan.inst.size() != 1) return fail(AMR_E_INVALID, "remesh works on single meshes");
  if (prm->max_blocks < h->plan.nleaf) return fail(AMR_E_CAPACITY, "max_blocks below the current leaf count");
  std::vector<double> S(S_host, S_host + h->plan.nleaf);
  return decide(h, S, prm, out, stats);
}

amr_status amr_remesh_apply(amr_mesh* nh, const double* Uold, double* Unew, void* stream) {
  amr_status rc = check_ready(nh, Unew);
  if (rc != AMR_OK) return rc;
  if (!Uold) return fail(AMR_E_INVALID, "null old state");
  if (nh->plan.migr.size() != size_t(nh->plan.nleaf)) return fail(AMR_E_STATE, "mesh was not made by amr_remesh_plan");
  hipError_t e = launch_migrate(dev_plan(nh), Uold, Unew, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? AMR_OK : hip_fail(e, "migrate");
}

amr_status amr_mesh_set_launch(amr_mesh* h, const amr_launch_t* c) {
  if (!h || !c) return fail(AMR_E_INVALID, "null argument");
  for (int a = 0; a < 3; a++)
    if (c->sweep_mode[a] != 0 && c->sweep_mode[a] != 1) return fail(AMR_E_INVALID, "sweep_mode must be 0 or 1");
  auto ok = [](int b) { return b >= 64 && b <= 1024 && b % 64 == 0; };
  if (!ok(c->sweep_block) || !ok(c->refresh_block) || !ok(c->reflux_block))
    return fail(AMR_E_INVALID, "workgroup sizes must be multiples of 64 in 64..1024");
  if (c->sweep_block > 256 || c->refresh_block > 256 || c->reflux_block > 256)
    return fail(AMR_E_INVALID, "workgroup sizes above 256 exceed the kernels' launch bounds");
  for (int a = 0; a < 3; a++) h->cfg.sweep_mode[a] = c->sweep_mode[a];
  h->cfg.sweep_block = c->sweep_block;
  h->cfg.refresh_block = c->refresh_block;
  h->cfg.reflux_block = c->reflux_block;
  return AMR_OK;
}

amr_status amr_mesh_get_launch(const amr_mesh* h, amr_launch_t* c) {
  if (!h || !c) return fail(AMR_E_INVALID, "null argument");
  for (int a = 0; a < 3; a++) c->sweep_mode[a] = h->cfg.sweep_mode[a];
  c->sweep_block = h->cfg.sweep_block;
  c->refresh_block = h->cfg.refresh_block;
  c->reflux_block = h->cfg.reflux_block;
  return AMR_OK;
}

amr_status amr_profile_enable(amr_mesh* h, int32_t on) {
  if (!h) return fail(AMR_E_INVALID, "null mesh");
  h->prof.release_all();
  h->prof.on = on != 0;
  return AMR_OK;
}

amr_status amr_profile_read(amr_mesh* h, double* ms_out, int64_t* launches_out) {
  if (!h || !ms_out || !launches_out) return fail(AMR_E_INVALID, "null argument");
  for (int p = 0; p < AMR_NPHASE; p++) {
    ms_out[p] = 0.0;
    launches_out[p] = 0;
  }
  for (auto& r : h->prof.recs) {
    hipError_t e = hipEventSynchronize(r.b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return hip_fail(e, "profile read");
    ms_out[r.phase] += double(ms);
    launches_out[r.phase] += 1;
  }
  h->prof.release_all();
  return AMR_OK;
}

struct amr_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

amr_status amr_graph_create(amr_mesh* h, double* U, double* dt, int64_t first_step, void* stream, amr_graph** out) {
  if (!out) return fail(AMR_E_INVALID, "null output");
  *out = nullptr;
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt) return fail(AMR_E_INVALID, "null dt pointer");
  if (!stream) return fail(AMR_E_INVALID, "graph capture needs a non-null stream");
  if (h->prof.on) return fail(AMR_E_STATE, "turn profiling off before capturing");
  hipStream_t st = static_cast<hipStream_t>(stream);
  amr_graph* g = new (std::nothrow) amr_graph();
  if (!g) return fail(AMR_E_NOMEM, "out of host memory");
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "begin capture");
  }
  const DevPlan P = dev_plan(h);
  // The first step's CFL reduction reads the state; the second step's is
  // accumulated by the first step and only finalized (as in amr_hydro_steps).
  double* const inplace[3] = {U, U, U};
  amr_status srs = AMR_OK;
  hipError_t e2 = launch_cfl(P, U, dt, h->cfg, st);
  if (e2 != hipSuccess) srs = hip_fail(e2, "cfl");
  if (srs == AMR_OK) srs = run_step_into(h, U, inplace, dt, first_step, st, nullptr, 1);
  if (srs == AMR_OK && (e2 = launch_cfl_finalize(P, dt, st)) != hipSuccess) srs = hip_fail(e2, "cfl");
  if (srs == AMR_OK) srs = run_step(h, U, dt, first_step + 1, st);
  e = hipStreamEndCapture(st, &g->graph);
  if (srs != AMR_OK || e != hipSuccess) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return srs != AMR_OK ? srs : hip_fail(e, "end capture");
  }
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return hip_fail(e, "instantiate");
  }
  *out = g;
  return AMR_OK;
}

amr_status amr_graph_launch(amr_graph* g, void* stream) {
  if (!g) return fail(AMR_E_INVALID, "null graph");
  hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? AMR_OK : hip_fail(e, "graph launch");
}

amr_status amr_graph_destroy(amr_graph* g) {
  if (!g) return AMR_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return AMR_OK;
}

namespace {

// The mg0 solver's grid: one instance whose leaves are all at level 0, periodic
// on every axis, with a coarsest level that fits one workgroup.
amr_status poisson_grid(const amr_mesh* h, int n[3]) {
  const Plan& p = h->plan;
  if (p.inst.size() != 1) return fail(AMR_E_INVALID, "the Poisson solver takes one mesh, not a batch");
  for (const Key& k : p.keys)
    if (k.l != 0) return fail(AMR_E_INVALID, "the Poisson solver needs a uniform mesh (all leaves at level 0)");
  const InstParams& ip = p.inst[0];
  for (int a = 0; a < 3; a++) {
    if (ip.bc[a] != AMR_BC_PERIODIC) return fail(AMR_E_INVALID, "the Poisson solver needs periodic boundaries");
    n[a] = ip.root[a] * p.N;
  }
  int sz[kMgMaxLevels][3];
  const int nl = mg_levels(n[0], n[1], n[2], sz);
  if (int64_t(sz[nl - 1][0]) * sz[nl - 1][1] * sz[nl - 1][2] > kMgCoarseMax)
    return fail(AMR_E_INVALID, "the Poisson solver's coarsest level exceeds 4096 cells (odd parts of the root extents too large)");
  return AMR_OK;
}

}  // namespace

namespace {

// The root grid of a single periodic mesh (refined or not) for the Poisson
// entries; *refined says whether any leaf lies below level 0.
amr_status poisson_root(const amr_mesh* h, int n[3], bool* refined) {
  const Plan& p = h->plan;
  if (p.inst.size() != 1) return fail(AMR_E_INVALID, "the Poisson solver takes one mesh, not a batch");
  *refined = false;
  for (const Key& k : p.keys) *refined = *refined || k.l != 0;
  const InstParams& ip = p.inst[0];
  for (int a = 0; a < 3; a++) {
    if (ip.bc[a] != AMR_BC_PERIODIC) return fail(AMR_E_INVALID, "the Poisson solver needs periodic boundaries");
    n[a] = ip.root[a] * p.N;
  }
  int sz[kMgMaxLevels][3];
  const int nl = mg_levels(n[0], n[1], n[2], sz);
  if (int64_t(sz[nl - 1][0]) * sz[nl - 1][1] * sz[nl - 1][2] > kMgCoarseMax)
    return fail(AMR_E_INVALID, "the Poisson solver's coarsest level exceeds 4096 cells (odd parts of the root extents too large)");
  return AMR_OK;
}

inline uint64_t pack_key(int l, int i, int j, int k) {
  return (uint64_t(l) << 60) | (uint64_t(k) << 40) | (uint64_t(j) << 20) | uint64_t(i);
}

// The hierarchy of mg0 on the octree: stage l (0 <= l < lmax) = the leaves
// coarser than l and every node of level l; stage lmax = the mesh.
amr_status build_composite(amr_mesh* h, const int n[3]) {
  if (h->comp) return AMR_OK;
  std::unique_ptr<CompositeMg> C(new (std::nothrow) CompositeMg());
  if (!C) return fail(AMR_E_NOMEM, "out of host memory");
  const Plan& top = h->plan;
  const Octree& T = *h->tree;
  const int N = top.N, M = N + 2 * kGhost;
  int lmax = 0;
  for (const Key& k : top.keys) lmax = std::max(lmax, int(k.l));
  C->lmax = lmax;
  C->plans.resize(size_t(lmax));
  C->nleaf.assign(size_t(lmax + 1), 0);
  std::vector<FlatMap<int32_t>> index(size_t(lmax + 1));
  for (int l = 0; l < lmax; l++) {
    std::vector<int32_t> keys;
    for (const Key& k : top.keys)
      if (k.l < l) keys.insert(keys.end(), {k.l, k.i, k.j, k.k});
    for (int kz = 0; kz < T.ext(l, 2); kz++)
      for (int ky = 0; ky < T.ext(l, 1); ky++)
        for (int kx = 0; kx < T.ext(l, 0); kx++)
          if (T.state(l, kx, ky, kz) != Octree::ABSENT) keys.insert(keys.end(), {int32_t(l), kx, ky, kz});
    C->trees.emplace_back(new Octree(T.desc()));
    std::string e = C->trees.back()->from_leaves(keys.data(), int64_t(keys.size() / 4));
    if (e.empty()) e = C->plans[size_t(l)].build({C->trees.back().get()});
    if (!e.empty()) return fail(AMR_E_BALANCE, "mg0 hierarchy stage " + std::to_string(l) + ": " + e);
  }
  for (int l = 0; l <= lmax; l++) {
    const Plan& P = l == lmax ? top : C->plans[size_t(l)];
    C->nleaf[size_t(l)] = P.nleaf;
    index[size_t(l)].reserve(size_t(P.nleaf));
    for (int64_t s = 0; s < P.nleaf; s++) {
      const Key& k = P.keys[size_t(s)];
      index[size_t(l)][pack_key(k.l, k.i, k.j, k.k)] = int32_t(s);
    }
  }
  auto find = [&](int stage, int l, int i, int j, int k) -> int32_t {
    const int32_t* v = index[size_t(stage)].find(pack_key(l, i, j, k));
    return v ? *v : -1;
  };
  C->rtask.resize(size_t(lmax));
  C->ptask.resize(size_t(lmax + 1));
  for (int l = 0; l < lmax; l++) {
    const Plan& P = C->plans[size_t(l)];
    for (int64_t s = 0; s < P.nleaf; s++) {
      const Key& k = P.keys[size_t(s)];
      MigrTask t{};
      const int32_t same = find(l + 1, k.l, k.i, k.j, k.k);
      if (same >= 0) {
        t.kind = MIGR_COPY;
        t.src[0] = same;
      } else {
        t.kind = MIGR_RESTRICT;
        for (int o = 0; o < 8; o++) {
          t.src[o] = find(l + 1, k.l + 1, 2 * k.i + (o & 1), 2 * k.j + ((o >> 1) & 1), 2 * k.k + (o >> 2));
          if (t.src[o] < 0) return fail(AMR_E_BALANCE, "mg0 hierarchy: missing child");
        }
      }
      C->rtask[size_t(l)].push_back(t);
    }
  }
  for (int l = 1; l <= lmax; l++) {
    const Plan& P = l == lmax ? top : C->plans[size_t(l)];
    for (int64_t s = 0; s < P.nleaf; s++) {
      const Key& k = P.keys[size_t(s)];
      MigrTask t{};
      const int32_t same = find(l - 1, k.l, k.i, k.j, k.k);
      if (same >= 0) {
        t.kind = MIGR_COPY;
        t.src[0] = same;
      } else {
        t.kind = MIGR_PROLONG;
        t.co = (k.i & 1) + 2 * (k.j & 1) + 4 * (k.k & 1);
        t.src[0] = find(l - 1, k.l - 1, k.i >> 1, k.j >> 1, k.k >> 1);
        if (t.src[0] < 0) return fail(AMR_E_BALANCE, "mg0 hierarchy: missing parent");
      }
      C->ptask[size_t(l)].push_back(t);
    }
  }
  auto al = [](int64_t v) { return (v + 255) / 256 * 256; };
  const int64_t M3 = int64_t(M) * M * M, N3 = int64_t(N) * N * N;
  int64_t o = 0;
  C->off_plan.assign(size_t(lmax + 1), 0);
  C->off_r.assign(size_t(lmax + 1), 0);
  C->off_p.assign(size_t(lmax + 1), 0);
  for (int l = 0; l < lmax; l++) {
    C->off_plan[size_t(l)] = o;
    o = al(o + C->plans[size_t(l)].off.total);
  }
  for (int l = 0; l <= lmax; l++) {
    C->off_r[size_t(l)] = o;
    if (l < lmax) o = al(o + int64_t(C->rtask[size_t(l)].size() * sizeof(MigrTask)));
    C->off_p[size_t(l)] = o;
    if (l >= 1) o = al(o + int64_t(C->ptask[size_t(l)].size() * sizeof(MigrTask)));
  }
  C->tables = o;
  C->off_x.assign(size_t(lmax + 1), 0);
  C->off_b.assign(size_t(lmax + 1), 0);
  C->off_L.assign(size_t(lmax + 1), 0);
  for (int l = 0; l <= lmax; l++) {
    const int64_t nb = C->nleaf[size_t(l)];
    C->off_x[size_t(l)] = o; o = al(o + nb * M3 * 8);
    C->off_b[size_t(l)] = o; o = al(o + nb * N3 * 8);
    C->off_L[size_t(l)] = o; o = al(o + nb * N3 * 8);
  }
  C->off_mg = o; o = al(o + mg_workspace_bytes(n[0], n[1], n[2]));
  C->off_parts = o; o = al(o + top.nleaf * 8);
  C->off_scal = o; o = al(o + 8 * 8);
  C->total = o;
  C->staging.assign(size_t(C->tables), 0);
  for (int l = 0; l < lmax; l++) {
    const Plan& P = C->plans[size_t(l)];
    std::memcpy(C->staging.data() + C->off_plan[size_t(l)], P.staging.data(), P.staging.size());
    std::memcpy(C->staging.data() + C->off_r[size_t(l)], C->rtask[size_t(l)].data(),
                C->rtask[size_t(l)].size() * sizeof(MigrTask));
  }
  for (int l = 1; l <= lmax; l++)
    std::memcpy(C->staging.data() + C->off_p[size_t(l)], C->ptask[size_t(l)].data(),
                C->ptask[size_t(l)].size() * sizeof(MigrTask));
  C->volume = 0.0;
  for (const Key& k : top.keys) C->volume += std::ldexp(double(N3), -3 * k.l);
  h->comp = std::move(C);
  return AMR_OK;
}

amr_status poisson_bytes(amr_mesh* h, int64_t* bytes) {
  int n[3];
  bool refined = false;
  amr_status rc = poisson_root(h, n, &refined);
  if (rc != AMR_OK) return rc;
  if (!refined) {
    *bytes = mg_workspace_bytes(n[0], n[1], n[2]);
    return AMR_OK;
  }
  rc = build_composite(h, n);
  if (rc != AMR_OK) return rc;
  *bytes = h->comp->total;
  return AMR_OK;
}

// The composite V-cycles (the hierarchy and its workspace layout built).
hipError_t composite_solve(amr_mesh* h, const int n[3], const double* f, double* phi, int ncycles, int nu1, int nu2,
                           double* resid, unsigned char* work, hipStream_t st) {
  const CompositeMg& C = *h->comp;
  const int lmax = C.lmax;
  const int N = h->plan.N;
  const int64_t N3 = int64_t(N) * N * N;
  hipError_t e = hipMemcpyAsync(work, C.staging.data(), size_t(C.tables), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  std::vector<DevPlan> SP(size_t(lmax + 1));
  std::vector<double*> X(size_t(lmax + 1)), B(size_t(lmax + 1)), L(size_t(lmax + 1));
  for (int l = 0; l <= lmax; l++) {
    SP[size_t(l)] = l == lmax ? dev_plan(h) : dev_plan_at(C.plans[size_t(l)], work + C.off_plan[size_t(l)]);
    X[size_t(l)] = reinterpret_cast<double*>(work + C.off_x[size_t(l)]);
    B[size_t(l)] = reinterpret_cast<double*>(work + C.off_b[size_t(l)]);
    L[size_t(l)] = reinterpret_cast<double*>(work + C.off_L[size_t(l)]);
  }
  double* parts = reinterpret_cast<double*>(work + C.off_parts);
  double* scal = reinterpret_cast<double*>(work + C.off_scal);
  auto op = [&](int kind, int l) {
    CzOp o;
    o.kind = kind;
    o.P = SP[size_t(l)];
    o.x = X[size_t(l)];
    o.b = B[size_t(l)];
    o.L = L[size_t(l)];
    o.parts = parts;
    o.scal = scal;
    return o;
  };
  auto operator_on = [&](int l, int col) {
    hipError_t r = launch_refresh_scalar(SP[size_t(l)], X[size_t(l)], st);
    if (r != hipSuccess) return r;
    CzOp o = op(CZ_OPERATOR, l);
    o.col = col;
    return cz_launch(o, st);
  };
  auto pass = [&](int l, int col) {
    hipError_t r = operator_on(l, col);
    if (r != hipSuccess) return r;
    CzOp o = op(CZ_UPDATE, l);
    o.col = col;
    return cz_launch(o, st);
  };
  auto residual = [&](int l) {
    hipError_t r = operator_on(l, -1);
    return r != hipSuccess ? r : cz_launch(op(CZ_RESID, l), st);
  };
  const double dx0 = 1.0 / double(int64_t(h->plan.inst[0].root[0]) * N);
  std::function<hipError_t(int)> vcycle = [&](int l) -> hipError_t {
    hipError_t r = hipSuccess;
    if (l == 0)
      return mg_vcycle_blocks(SP[0], n[0], n[1], n[2], dx0, B[0], X[0], nu1, nu2, work + C.off_mg, st);
    for (int k = 0; k < nu1 && r == hipSuccess; k++) {
      r = pass(l, 0);
      if (r == hipSuccess) r = pass(l, 1);
    }
    if (r == hipSuccess) r = residual(l);
    if (r == hipSuccess) {
      CzOp o = op(CZ_RESTRICT, l - 1);
      o.L = L[size_t(l)];
      o.tasks = reinterpret_cast<const MigrTask*>(work + C.off_r[size_t(l - 1)]);
      r = cz_launch(o, st);
    }
    if (r == hipSuccess) r = cz_launch(op(CZ_ZERO, l - 1), st);
    if (r == hipSuccess) r = vcycle(l - 1);
    if (r == hipSuccess) r = launch_refresh_scalar(SP[size_t(l - 1)], X[size_t(l - 1)], st);
    if (r == hipSuccess) {
      CzOp o = op(CZ_PROLONG, l);
      o.e = X[size_t(l - 1)];
      o.tasks = reinterpret_cast<const MigrTask*>(work + C.off_p[size_t(l)]);
      r = cz_launch(o, st);
    }
    for (int k = 0; k < nu2 && r == hipSuccess; k++) {
      r = pass(l, 0);
      if (r == hipSuccess) r = pass(l, 1);
    }
    return r;
  };
  if (f != B[size_t(lmax)]) {
    e = hipMemcpyAsync(B[size_t(lmax)], f, size_t(h->plan.nleaf * N3 * 8), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  CzOp mo = op(CZ_MEAN_SUB, lmax);
  mo.scale = 1.0 / C.volume;
  if ((e = cz_launch(mo, st)) != hipSuccess) return e;
  if ((e = cz_launch(op(CZ_ZERO, lmax), st)) != hipSuccess) return e;
  CzOp ci = op(CZ_COPY_IN, lmax);
  ci.src = phi;
  if ((e = cz_launch(ci, st)) != hipSuccess) return e;
  auto norm = [&](int c) {
    if (!resid) return hipSuccess;
    hipError_t r = residual(lmax);
    if (r != hipSuccess) return r;
    CzOp o = op(CZ_NORM, lmax);
    o.scal = resid + c;
    return cz_launch(o, st);
  };
  if ((e = norm(0)) != hipSuccess) return e;
  for (int c = 0; c < ncycles; c++) {
    if ((e = vcycle(lmax)) != hipSuccess) return e;
    if ((e = norm(c + 1)) != hipSuccess) return e;
  }
  CzOp mp = op(CZ_MEAN_PADDED, lmax);
  mp.scale = 1.0 / C.volume;
  mp.scal = scal + 1;
  if ((e = cz_launch(mp, st)) != hipSuccess) return e;
  CzOp co = op(CZ_COPY_OUT, lmax);
  co.dst = phi;
  co.scal = scal + 1;
  return cz_launch(co, st);
}

amr_status poisson_run(amr_mesh* h, const double* f, double* phi, int32_t ncycles, int32_t nu1, int32_t nu2,
                       double* resid, void* work, int64_t work_cap, void* stream) {
  int n[3];
  bool refined = false;
  amr_status rc = poisson_root(h, n, &refined);
  if (rc != AMR_OK) return rc;
  int64_t need = 0;
  rc = poisson_bytes(h, &need);
  if (rc != AMR_OK) return rc;
  if (work_cap >= 0 && need > work_cap)
    return fail(AMR_E_CAPACITY, "grid of " + std::to_string(n[0]) + "x" + std::to_string(n[1]) + "x" +
                                    std::to_string(n[2]) + " needs a " + std::to_string(need) +
                                    "-byte workspace, above the fixed buffer's " + std::to_string(work_cap) +
                                    " bytes (use amr_poisson_solve)");
  const Plan& p = h->plan;
  const double dx = 1.0 / double(int64_t(p.inst[0].root[0]) * p.N);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = timed(h, AMR_PHASE_POISSON, st, [&] {
    if (refined)
      return composite_solve(h, n, f, phi, ncycles, nu1, nu2, resid, static_cast<unsigned char*>(work), st);
    return mg_solve(dev_plan(h), n[0], n[1], n[2], dx, f, nullptr, 0.0, phi, ncycles, nu1, nu2, resid, work, st);
  });
  return e == hipSuccess ? AMR_OK : hip_fail(e, "poisson");
}

// Self-gravity pieces on a refined mesh (composite layout of work): the
// solve for four_pi_G times U's density, and a half kick with -grad(phi).
hipError_t composite_gravity_solve(amr_mesh* h, const int n[3], const double* U, double four_pi_G, double* phi,
                                   int ncycles, int nu1, int nu2, unsigned char* work, hipStream_t st) {
  const CompositeMg& C = *h->comp;
  double* b = reinterpret_cast<double*>(work + C.off_b[size_t(C.lmax)]);
  CzOp o;
  o.kind = CZ_DENSITY;
  o.P = dev_plan(h);
  o.U = const_cast<double*>(U);
  o.b = b;
  o.fpg = four_pi_G;
  hipError_t e = cz_launch(o, st);
  if (e != hipSuccess) return e;
  return composite_solve(h, n, b, phi, ncycles, nu1, nu2, nullptr, work, st);
}

hipError_t composite_kick(amr_mesh* h, double* U, const double* phi, const double* dt, double scale,
                          unsigned char* work, hipStream_t st) {
  const CompositeMg& C = *h->comp;
  CzOp o;
  o.P = dev_plan(h);
  o.x = reinterpret_cast<double*>(work + C.off_x[size_t(C.lmax)]);
  o.kind = CZ_ZERO;
  hipError_t e = cz_launch(o, st);
  o.kind = CZ_COPY_IN;
  o.src = phi;
  if (e == hipSuccess) e = cz_launch(o, st);
  if (e == hipSuccess) e = launch_refresh_scalar(o.P, o.x, st);
  o.kind = CZ_KICK;
  o.U = U;
  o.dt = dt;
  o.scale = scale;
  if (e == hipSuccess) e = cz_launch(o, st);
  return e;
}

}  // namespace

amr_status amr_poisson_workspace_bytes(const amr_mesh* h, int64_t* bytes) {
  if (!h || !bytes) return fail(AMR_E_INVALID, "null argument");
  return poisson_bytes(const_cast<amr_mesh*>(h), bytes);
}

amr_status amr_poisson_solve(amr_mesh* h, const double* f, double* phi, int32_t ncycles, int32_t nu1, int32_t nu2,
                             double* resid, void* work, void* stream) {
  if (!h) return fail(AMR_E_INVALID, "null mesh");
  if (!h->ws) return fail(AMR_E_STATE, "no workspace uploaded");
  if (!f || !phi || !work) return fail(AMR_E_INVALID, "null argument");
  if (ncycles < 0 || nu1 < 0 || nu2 < 0 || nu1 > 64 || nu2 > 64)
    return fail(AMR_E_INVALID, "ncycles must be >= 0 and nu1, nu2 in [0, 64]");
  return poisson_run(h, f, phi, ncycles, nu1, nu2, resid, work, -1, stream);
}

amr_status amr_poisson_solve_static(amr_mesh* h, const double* f, double* phi, int32_t ncycles, int32_t nu1,
                                    int32_t nu2, double* resid, void* stream) {
  if (!h) return fail(AMR_E_INVALID, "null mesh");
  if (!h->ws) return fail(AMR_E_STATE, "no workspace uploaded");
  if (!f || !phi) return fail(AMR_E_INVALID, "null argument");
  if (ncycles < 0 || nu1 < 0 || nu2 < 0 || nu1 > 64 || nu2 > 64)
    return fail(AMR_E_INVALID, "ncycles must be >= 0 and nu1, nu2 in [0, 64]");
  int64_t need = 0;
  amr_status rc = poisson_bytes(h, &need);
  if (rc != AMR_OK) return rc;
  if (need > kMgStaticScratchBytes) return poisson_run(h, f, phi, ncycles, nu1, nu2, resid, nullptr,
                                                       kMgStaticScratchBytes, stream);
  void* work = nullptr;
  hipError_t e = mg_static_scratch(&work);
  if (e != hipSuccess) return hip_fail(e, "poisson fixed workspace");
  return poisson_run(h, f, phi, ncycles, nu1, nu2, resid, work, kMgStaticScratchBytes, stream);
}

amr_status amr_hydro_step_gravity(amr_mesh* h, double* U, double* dt, int64_t step_index, double four_pi_G,
                                  double* phi, int32_t phi_current, int32_t ncycles, int32_t nu1, int32_t nu2,
                                  void* work, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt || !phi || !work) return fail(AMR_E_INVALID, "null argument");
  if (!std::isfinite(four_pi_G)) return fail(AMR_E_INVALID, "four_pi_G must be finite");
  if (ncycles < 0 || nu1 < 0 || nu2 < 0 || nu1 > 64 || nu2 > 64)
    return fail(AMR_E_INVALID, "ncycles must be >= 0 and nu1, nu2 in [0, 64]");
  int n[3];
  bool refined = false;
  rc = poisson_root(h, n, &refined);
  if (rc != AMR_OK) return rc;
  if (refined) {
    int64_t need = 0;
    rc = poisson_bytes(h, &need);
    if (rc != AMR_OK) return rc;
  }
  const Plan& p = h->plan;
  const double dx = 1.0 / double(int64_t(p.inst[0].root[0]) * p.N);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  unsigned char* wb = static_cast<unsigned char*>(work);
  auto solve = [&] {
    return timed(h, AMR_PHASE_POISSON, st, [&] {
      if (refined) return composite_gravity_solve(h, n, U, four_pi_G, phi, ncycles, nu1, nu2, wb, st);
      return mg_solve(P, n[0], n[1], n[2], dx, nullptr, U, four_pi_G, phi, ncycles, nu1, nu2, nullptr, work, st);
    });
  };
  auto kick = [&](bool after_solve) {
    return timed(h, AMR_PHASE_POISSON, st, [&] {
      if (refined) return composite_kick(h, U, phi, dt, 1.0, wb, st);
      return mg_kick(P, n[0], n[1], n[2], dx, U, phi, dt, 1.0, work, st, 0, nullptr, 0.0, after_solve);
    });
  };
  hipError_t e = hipSuccess;
  if (!phi_current) e = solve();
  if (e == hipSuccess) e = timed(h, AMR_PHASE_CFL, st, [&] { return launch_cfl(P, U, dt, h->cfg, st); });
  if (e == hipSuccess) e = kick(!phi_current);
  if (e != hipSuccess) return hip_fail(e, "gravity");
  rc = run_step(h, U, dt, step_index, st);
  if (rc != AMR_OK) return rc;
  e = solve();
  if (e == hipSuccess) e = kick(true);
  return e == hipSuccess ? AMR_OK : hip_fail(e, "gravity");
}

amr_status amr_hydro_step_gravity_comoving(amr_mesh* h, double* U, const double* dt, int64_t step_index, double a0,
                                           double a_mid, double a1, double hubble, double four_pi_G, double* phi,
                                           int32_t phi_current, int32_t ncycles, int32_t nu1, int32_t nu2,
                                           void* work, void* stream) {
  amr_status rc = check_ready(h, U);
  if (rc != AMR_OK) return rc;
  if (!dt || !phi || !work) return fail(AMR_E_INVALID, "null argument");
  for (double a : {a0, a_mid, a1})
    if (!(a > 0.0) || !std::isfinite(a)) return fail(AMR_E_INVALID, "expansion factors must be positive and finite");
  if (!std::isfinite(hubble) || !std::isfinite(four_pi_G))
    return fail(AMR_E_INVALID, "expansion rate and four_pi_G must be finite");
  if (ncycles < 0 || nu1 < 0 || nu2 < 0 || nu1 > 64 || nu2 > 64)
    return fail(AMR_E_INVALID, "ncycles must be >= 0 and nu1, nu2 in [0, 64]");
  int n[3];
  rc = poisson_grid(h, n);
  if (rc != AMR_OK) return rc;
  const Plan& p = h->plan;
  const double dx = 1.0 / double(int64_t(p.inst[0].root[0]) * p.N);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevPlan P = dev_plan(h);
  auto solve = [&] {
    return timed(h, AMR_PHASE_POISSON, st, [&] {
      return mg_solve(P, n[0], n[1], n[2], dx, nullptr, U, four_pi_G, phi, ncycles, nu1, nu2, nullptr, work, st);
    });
  };
  // the kicks carry the expansion sources in the same pass: the first kick
  // is followed by the first half of the sources, the last kick preceded by
  // the second half (the solve between them reads only the density, which
  // the sources leave alone)
  double* half = nullptr;
  auto kick = [&](double a, int exp, bool after_solve) {
    const double scale = 1.0 / (a * a);
    return timed(h, AMR_PHASE_POISSON, st, [&] {
      return mg_kick(P, n[0], n[1], n[2], dx, U, phi, dt, scale, work, st, exp, half, hubble, after_solve);
    });
  };
  hipError_t e = hipSuccess;
  if (!phi_current) e = solve();
  if (e == hipSuccess) {
    half = mg_half_dt(dt, work, n[0], n[1], n[2], st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = kick(a0, 1, !phi_current);
  if (e == hipSuccess) e = launch_scale_dt(P, dt, a_mid, st);
  if (e != hipSuccess) return hip_fail(e, "gravity");
  rc = run_step(h, U, P.dte, step_index, st);
  if (rc != AMR_OK) return rc;
  e = solve();
  if (e == hipSuccess) e = kick(a1, 2, true);
  return e == hipSuccess ? AMR_OK : hip_fail(e, "gravity");
}

amr_status amr_arith_selftest(uint64_t seed, int64_t n, uint64_t* counts, void* stream) {
  if (!counts) return fail(AMR_E_INVALID, "null counts");
  if (n < 0 || n > (int64_t(1) << 40)) return fail(AMR_E_INVALID, "operand count out of range");
  hipError_t e = launch_arith_check(seed, n, reinterpret_cast<unsigned long long*>(counts),
                                    static_cast<hipStream_t>(stream));
  return e == hipSuccess ? AMR_OK : hip_fail(e, "arithmetic self-test");
}

const char* amr_last_error(void) { return g_err.c_str(); }

}  // extern "C"
