// mesh.cpp -- octree, 2:1 balance and plan tables (host side).
//
// The array-of-octrees of the paper (Sec. II-B): a root array of octrees, a
// Block per node, leaves carry data.  Refinement keeps neighbouring leaves
// (across faces, edges and corners, periodic wrap included) within one level
// of each other, which bounds every ghost cell's source to one level of
// difference and lets the two-phase refresh read only copied or restricted
// values when it prolongs.
#include "mesh.hpp"

#include <algorithm>
#include <cstring>
#include <memory>
#include <stdexcept>

namespace amr {

InstParams make_inst_params(const MeshDesc& d) {
  InstParams p{};
  p.gamma = d.gamma;
  p.gm1 = d.gamma - 1.0;
  p.inv_gm1 = 1.0 / (d.gamma - 1.0);
  p.g_gm1 = d.gamma / (d.gamma - 1.0);
  p.g1 = (d.gamma + 1.0) / (2.0 * d.gamma);
  p.rho_floor = d.rho_floor;
  p.p_floor = d.p_floor;
  p.cfl = d.cfl;
  p.sixth = 1.0 / 6.0;
  p.two3 = 2.0 / 3.0;
  for (int a = 0; a < 3; a++) {
    p.root[a] = d.root[a];
    p.bc[a] = d.bc[a];
  }
  p.iters = d.iters;
  p.de = d.de;
  p.eta1 = d.eta1;
  p.eta2 = d.eta2;
  return p;
}

Octree::Octree(const MeshDesc& d) : d_(d) {
  for (int k = 0; k < d.root[2]; k++)
    for (int j = 0; j < d.root[1]; j++)
      for (int i = 0; i < d.root[0]; i++) node_[pack(0, i, j, k)] = LEAF;
}

uint8_t Octree::state(int l, int i, int j, int k) const {
  const uint8_t* v = node_.find(pack(l, i, j, k));
  return v ? *v : ABSENT;
}

bool Octree::wrap(int l, int ax, int& v) const {
  const int e = ext(l, ax);
  if (v >= 0 && v < e) return true;
  if (d_.bc[ax] != 0) return false;
  v = ((v % e) + e) % e;
  return true;
}

void Octree::refine(int l, int i, int j, int k) {
  node_[pack(l, i, j, k)] = REFINED;
  for (int c = 0; c < 8; c++)
    node_[pack(l + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + (c >> 2))] = LEAF;
}

void Octree::unrefine(int l, int i, int j, int k) {
  node_[pack(l, i, j, k)] = LEAF;
  for (int c = 0; c < 8; c++) node_.erase(pack(l + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + (c >> 2)));
}

std::string Octree::refine_list(const int32_t* keys, int64_t n) {
  for (int64_t r = 0; r < n; r++) {
    const int32_t* e = keys + 4 * r;
    const int l = e[0];
    if (l < 0 || l >= d_.max_level) return "refine entry level out of range";
    for (int a = 0; a < 3; a++)
      if (e[1 + a] < 0 || e[1 + a] >= ext(l, a)) return "refine entry key out of range";
    // walk down from the root, splitting leaves on the way
    for (int a = 0; a <= l; a++) {
      const int s = l - a;
      const int i = e[1] >> s, j = e[2] >> s, k = e[3] >> s;
      if (state(a, i, j, k) == LEAF) refine(a, i, j, k);
    }
  }
  balance();
  return "";
}

// Level-by-level balance, finest first: a leaf at level l needs every
// neighbouring position's level-(l-1) node to exist; creating it only adds
// nodes at levels <= l-1, which are handled when their level comes.
void Octree::balance() {
  for (int l = d_.max_level; l >= 2; l--) {
    std::vector<Key> level_leaves;
    node_.for_each([&](uint64_t p, uint8_t st) {
      if (st == LEAF && int(p >> 60) == l)
        level_leaves.push_back({l, int(p & 0xFFFFF), int((p >> 20) & 0xFFFFF), int((p >> 40) & 0xFFFFF)});
    });
    for (const Key& lf : level_leaves) {
      for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
          for (int dx = -1; dx <= 1; dx++) {
            if (!dx && !dy && !dz) continue;
            int q[3] = {lf.i + dx, lf.j + dy, lf.k + dz};
            bool in = true;
            for (int a = 0; a < 3; a++) in = in && wrap(l, a, q[a]);
            if (!in) continue;
            const int t = l - 1;  // target level that must exist
            for (int a = 0; a < t; a++) {
              const int s = l - a;
              const int i = q[0] >> s, j = q[1] >> s, k = q[2] >> s;
              if (state(a, i, j, k) == LEAF) refine(a, i, j, k);
            }
          }
    }
  }
}

std::string Octree::check_balance() const {
  bool ok = true;
  node_.for_each([&](uint64_t p, uint8_t st) {
    if (!ok || st != LEAF) return;
    const int l = int(p >> 60);
    if (l < 2) return;
    const int i = int(p & 0xFFFFF), j = int((p >> 20) & 0xFFFFF), k = int((p >> 40) & 0xFFFFF);
    for (int dz = -1; dz <= 1; dz++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
          if (!dx && !dy && !dz) continue;
          int q[3] = {i + dx, j + dy, k + dz};
          bool in = true;
          for (int a = 0; a < 3; a++) in = in && wrap(l, a, q[a]);
          if (!in) continue;
          if (state(l - 1, q[0] >> 1, q[1] >> 1, q[2] >> 1) == ABSENT) ok = false;
        }
  });
  return ok ? "" : "leaves violate 2:1 balance";
}

std::string Octree::from_leaves(const int32_t* keys, int64_t n) {
  node_.clear();
  for (int64_t s = 0; s < n; s++) {
    const int32_t* e = keys + 4 * s;
    const int l = e[0];
    if (l < 0 || l > d_.max_level) return "leaf level out of range";
    for (int a = 0; a < 3; a++)
      if (e[1 + a] < 0 || e[1 + a] >= ext(l, a)) return "leaf key out of range";
    auto& st = node_[pack(l, e[1], e[2], e[3])];
    if (st != ABSENT) return "duplicate or nested leaf";
    st = LEAF;
    for (int a = l - 1; a >= 0; a--) {
      const int s2 = l - a;
      auto& pa = node_[pack(a, e[1] >> s2, e[2] >> s2, e[3] >> s2)];
      if (pa == LEAF) return "leaf inside another leaf";
      pa = REFINED;
    }
  }
  for (int k = 0; k < d_.root[2]; k++)
    for (int j = 0; j < d_.root[1]; j++)
      for (int i = 0; i < d_.root[0]; i++)
        if (state(0, i, j, k) == ABSENT) return "leaves do not cover the domain";
  const char* err = nullptr;
  node_.for_each([&](uint64_t p, uint8_t st) {
    if (err || st != REFINED) return;
    const int l = int(p >> 60);
    const int i = int(p & 0xFFFFF), j = int((p >> 20) & 0xFFFFF), k = int((p >> 40) & 0xFFFFF);
    if (l + 1 > d_.max_level) {
      err = "refined node at the deepest level";
      return;
    }
    for (int c = 0; c < 8; c++)
      if (state(l + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + (c >> 2)) == ABSENT) {
        err = "leaves do not tile the domain";
        return;
      }
  });
  if (err) return err;
  return check_balance();
}

void Octree::dfs(int l, int i, int j, int k, std::vector<Key>& out) const {
  const uint8_t s = state(l, i, j, k);
  if (s == LEAF) {
    out.push_back({l, i, j, k});
    return;
  }
  for (int c = 0; c < 8; c++) dfs(l + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + (c >> 2), out);
}

std::vector<Key> Octree::leaves() const {
  std::vector<Key> out;
  for (int k = 0; k < d_.root[2]; k++)
    for (int j = 0; j < d_.root[1]; j++)
      for (int i = 0; i < d_.root[0]; i++) dfs(0, i, j, k, out);
  return out;
}

// ---------------------------------------------------------------------------

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

std::string Plan::build(const std::vector<const Octree*>& meshes) {
  if (meshes.empty()) return "no meshes";
  N = meshes[0]->desc().N;
  M = N + 2 * kGhost;
  nf = meshes[0]->desc().de ? kFieldsDE : kFields;
  inst.clear(); blocks.clear(); nbr.clear(); fine.clear(); p2list.clear(); p2task.clear(); p2wave.clear(); faceslot.clear();
  keys.clear();
  std::vector<int32_t> p2k[3];  // phase-2 tasks by kind, merged below
  if (!migr.empty() && meshes.size() != 1) return "migration tables belong to single-mesh plans";
  for (auto& r : reflux) r.clear();
  nslots = 0;
  std::vector<int64_t> first;
  for (int m = 0; m < int(meshes.size()); m++) {
    const Octree& T = *meshes[m];
    if (T.desc().N != N) return "all meshes of a plan need the same block size";
    if ((T.desc().de ? kFieldsDE : kFields) != nf) return "all meshes of a plan need the same fields (dual energy on or off)";
    InstParams ip = make_inst_params(T.desc());
    ip.first_leaf = int64_t(blocks.size());
    const std::vector<Key> lv = T.leaves();
    ip.n_leaf = int64_t(lv.size());
    inst.push_back(ip);
    for (const Key& k : lv) {
      BlockInfo b{};
      b.level = k.l; b.i = k.i; b.j = k.j; b.k = k.k; b.inst = m;
      blocks.push_back(b);
      keys.push_back(k);
    }
  }
  nleaf = int64_t(blocks.size());
  // leaf id lookup per instance
  std::vector<FlatMap<int32_t>> id(meshes.size());
  for (size_t m = 0; m < meshes.size(); m++) id[m].reserve(size_t(inst[m].n_leaf));
  auto pk = [](int l, int i, int j, int k) {
    return (uint64_t(l) << 60) | (uint64_t(k) << 40) | (uint64_t(j) << 20) | uint64_t(i);
  };
  for (int64_t s = 0; s < nleaf; s++) {
    const BlockInfo& b = blocks[s];
    id[b.inst][pk(b.level, b.i, b.j, b.k)] = int32_t(s);
  }
  nbr.assign(size_t(27 * nleaf), Nbr{-1, -1});
  faceslot.assign(size_t(6 * nleaf), -1);
  for (int64_t s = 0; s < nleaf; s++) {
    const BlockInfo& b = blocks[s];
    const Octree& T = *meshes[b.inst];
    const int l = b.level;
    const int key[3] = {b.i, b.j, b.k};
    bool coarse_nbr = false;
    uint8_t nst[27];  // state of the node at each neighbour position (outflow: this leaf)
    nst[13] = Octree::LEAF;
    for (int code = 0; code < 27; code++) {
      if (code == 13) continue;
      const int sd[3] = {code % 3 - 1, (code / 3) % 3 - 1, code / 9 - 1};
      int q[3];
      for (int a = 0; a < 3; a++) {
        q[a] = key[a] + sd[a];
        if (!T.wrap(l, a, q[a])) q[a] = key[a];  // outflow: clamp to this block's slab
      }
      const uint8_t st = T.state(l, q[0], q[1], q[2]);
      nst[code] = st;
      Nbr& e = nbr[size_t(27 * s + code)];
      if (st == Octree::LEAF) {
        e.kind = NBR_COPY;
        const int32_t* it = id[b.inst].find(pk(l, q[0], q[1], q[2]));
        if (!it) return "leaf without a storage slot";
        e.id = *it;
      } else if (st == Octree::REFINED) {
        e.kind = NBR_FINE;
        e.id = int32_t(fine.size() / 8);
        for (int c = 0; c < 8; c++) {
          const int co[3] = {c & 1, (c >> 1) & 1, c >> 2};
          const int32_t* it = id[b.inst].find(pk(l + 1, 2 * q[0] + co[0], 2 * q[1] + co[1], 2 * q[2] + co[2]));
          fine.push_back(it ? *it : -1);
          // The ghost box of direction sd reads the children on the near
          // side along each axis with sd != 0 and both along sd == 0: those
          // touch this leaf, so balance makes them leaves.  Checked here
          // because the restriction kernel indexes them without a test.
          bool read = true;
          for (int a = 0; a < 3; a++) read = read && (sd[a] == 0 || co[a] == (sd[a] < 0 ? 1 : 0));
          if (read && fine.back() < 0) return "restriction source is not a leaf: mesh not balanced";
        }
      } else {
        const int32_t* it = l > 0 ? id[b.inst].find(pk(l - 1, q[0] >> 1, q[1] >> 1, q[2] >> 1)) : nullptr;
        if (!it) return "neighbour two levels coarser: mesh not balanced";
        e.kind = NBR_COARSE;
        e.id = *it;
        coarse_nbr = true;
        const int kind = (sd[0] != 0) + (sd[1] != 0) + (sd[2] != 0) - 1;  // 0 face, 1 edge, 2 corner
        p2k[kind].push_back(int32_t(s));
        p2k[kind].push_back(int32_t(code));
      }
    }
    if (coarse_nbr) p2list.push_back(int32_t(s));
    // coarse-fine faces get flux slots (a face on an outflow boundary saw
    // this leaf itself above, a leaf: no slot)
    for (int dir = 0; dir < 3; dir++)
      for (int side = 0; side < 2; side++) {
        const int code = 13 + (side ? 1 : -1) * (dir == 0 ? 1 : (dir == 1 ? 3 : 9));
        if (nst[code] != Octree::LEAF) faceslot[size_t(6 * s + 2 * dir + side)] = int32_t(nslots++);
      }
  }
  has_p2 = !p2list.empty();
  for (int k = 0; k < 3; k++) {
    np2t[k] = int64_t(p2k[k].size() / 2);
    p2task.insert(p2task.end(), p2k[k].begin(), p2k[k].end());
  }
  // the waves in leaf order (each kind's list is in leaf order: merge them)
  {
    int64_t first[3] = {0, np2t[0], np2t[0] + np2t[1]}, at[3] = {0, 0, 0};
    for (;;) {
      int k = -1;
      for (int q = 0; q < 3; q++)
        if (at[q] < np2t[q] && (k < 0 || p2k[q][size_t(2 * at[q])] < p2k[k][size_t(2 * at[k])])) k = q;
      if (k < 0) break;
      const int64_t row = first[k] + at[k]++;
      if (row >= (int64_t(1) << (31 - kP2SubBits))) return "too many phase-2 tasks";
      for (int w = 0; w < p2_waves(N, k); w++) p2wave.push_back(int32_t((row << kP2SubBits) | w));
    }
  }
  // reflux tasks: coarse side of each coarse-fine face
  for (int64_t s = 0; s < nleaf; s++) {
    const BlockInfo& b = blocks[s];
    const Octree& T = *meshes[b.inst];
    const int l = b.level;
    const int key[3] = {b.i, b.j, b.k};
    for (int dir = 0; dir < 3; dir++) {
      const int A = dir == 0 ? 1 : 0, B = dir == 2 ? 1 : 2;
      for (int side = 0; side < 2; side++) {
        const int32_t slot = faceslot[size_t(6 * s + 2 * dir + side)];
        if (slot < 0) continue;
        int q[3] = {key[0], key[1], key[2]};
        q[dir] += side ? 1 : -1;
        T.wrap(l, dir, q[dir]);
        if (T.state(l, q[0], q[1], q[2]) != Octree::REFINED) continue;
        RefluxTask t{};
        t.leaf = int32_t(s);
        t.side = side;
        t.slot_c = slot;
        for (int hB = 0; hB < 2; hB++)
          for (int hA = 0; hA < 2; hA++) {
            int c[3];
            c[dir] = 2 * q[dir] + (side ? 0 : 1);
            c[A] = 2 * key[A] + hA;
            c[B] = 2 * key[B] + hB;
            const int32_t* it = id[b.inst].find(pk(l + 1, c[0], c[1], c[2]));
            if (!it) return "refined face neighbour without leaf children";
            const int32_t fslot = faceslot[size_t(6 * *it + 2 * dir + (1 - side))];
            if (fslot < 0) return "fine face without a flux slot";
            t.slot_f[hA + 2 * hB] = fslot;
          }
        reflux[dir].push_back(t);
        blocks[size_t(s)].rflx |= 1 << (2 * dir + side);
      }
    }
  }
  // workspace layout
  int64_t o = 0;
  const int64_t ninst = int64_t(inst.size());
  off.inst = o; o = align256(o + ninst * int64_t(sizeof(InstParams)));
  off.blocks = o; o = align256(o + nleaf * int64_t(sizeof(BlockInfo)));
  off.nbr = o; o = align256(o + int64_t(nbr.size() * sizeof(Nbr)));
  off.fine = o; o = align256(o + int64_t(fine.size() * sizeof(int32_t)));
  off.p2list = o; o = align256(o + int64_t(p2list.size() * sizeof(int32_t)));
  off.p2task = o; o = align256(o + int64_t(p2task.size() * sizeof(int32_t)));
  off.p2wave = o; o = align256(o + int64_t(p2wave.size() * sizeof(int32_t)));
  off.faceslot = o; o = align256(o + int64_t(faceslot.size() * sizeof(int32_t)));
  for (int d = 0; d < 3; d++) {
    off.reflux[d] = o;
    o = align256(o + int64_t(reflux[d].size() * sizeof(RefluxTask)));
  }
  off.acc = o; o = align256(o + ninst * 8);
  off.lacc = o; o = align256(o + nleaf * kCflSlots * 8);
  off.dte = o; o = align256(o + ninst * 8);
  off.counters = o; o = align256(o + 8);
  off.ind = o; o = align256(o + nleaf * 8);
  off.migr = o; o = align256(o + int64_t(migr.size() * sizeof(MigrTask)));
  off.reloc = o; o = align256(o + int64_t(reloc.size() * sizeof(Reloc)));
  off.reloc_child = o; o = align256(o + int64_t(reloc_child.size() * sizeof(int32_t)));
  off.faces = o; o = align256(o + nslots * int64_t(nf) * N * N * 8);
  off.total = o;
  staging.assign(size_t(off.faces), 0);
  auto put = [&](int64_t at, const void* src, size_t bytes) {
    if (bytes) std::memcpy(staging.data() + at, src, bytes);
  };
  put(off.inst, inst.data(), inst.size() * sizeof(InstParams));
  put(off.blocks, blocks.data(), blocks.size() * sizeof(BlockInfo));
  put(off.nbr, nbr.data(), nbr.size() * sizeof(Nbr));
  put(off.fine, fine.data(), fine.size() * sizeof(int32_t));
  put(off.p2list, p2list.data(), p2list.size() * sizeof(int32_t));
  put(off.p2task, p2task.data(), p2task.size() * sizeof(int32_t));
  put(off.p2wave, p2wave.data(), p2wave.size() * sizeof(int32_t));
  put(off.faceslot, faceslot.data(), faceslot.size() * sizeof(int32_t));
  for (int d = 0; d < 3; d++) put(off.reflux[d], reflux[d].data(), reflux[d].size() * sizeof(RefluxTask));
  put(off.migr, migr.data(), migr.size() * sizeof(MigrTask));
  put(off.reloc, reloc.data(), reloc.size() * sizeof(Reloc));
  put(off.reloc_child, reloc_child.data(), reloc_child.size() * sizeof(int32_t));
  // dt accumulators start at +inf (bit pattern of a positive double)
  const uint64_t inf_bits = 0x7FF0000000000000ull;
  for (int64_t m = 0; m < ninst; m++) put(off.acc + 8 * m, &inf_bits, 8);
  return "";
}

// ---------------------------------------------------------------------------
// Remesh decisions.  Reading of the refinement rule (the paper names the
// Refine plug-in, not a criterion): leaves with S > refine_slope below the
// deepest level are candidates, taken in (S descending, then level, z, y, x)
// order; each is refined together with the minimal refinement restoring 2:1
// balance, accepted only if every node that closure refines was a leaf before
// this remesh (one level per remesh) and the leaf count stays <= max_blocks,
// else refused.  Then, finer parents first (ties by z, y, x), each octet of
// leaves that were leaves before and all have S < coarsen_slope merges if the
// merged leaf touches no leaf two levels finer.  Here the closure is a local
// ripple from the refined node with an undo journal.

namespace {
uint64_t pk4(int l, int i, int j, int k) {
  return (uint64_t(l) << 60) | (uint64_t(k) << 40) | (uint64_t(j) << 20) | uint64_t(i);
}
}  // namespace

RemeshResult remesh_decide(const Octree& old, const Plan& op, const std::vector<double>& S, double refine_slope,
                           double coarsen_slope, int64_t max_blocks) {
  RemeshResult res;
  res.tree.reset(new Octree(old));
  Octree& T = *res.tree;
  const MeshDesc& d = old.desc();
  FlatMap<int32_t> old_id;
  old_id.reserve(size_t(op.nleaf));
  for (int64_t s = 0; s < op.nleaf; s++) {
    const Key& k = op.keys[size_t(s)];
    old_id[pk4(k.l, k.i, k.j, k.k)] = int32_t(s);
  }
  int64_t leaves = op.nleaf;
  struct Cand {
    double S;
    Key k;
  };
  std::vector<Cand> cand;
  for (int64_t s = 0; s < op.nleaf; s++)
    if (S[size_t(s)] > refine_slope && op.keys[size_t(s)].l < d.max_level) cand.push_back({S[size_t(s)], op.keys[size_t(s)]});
  std::sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
    if (a.S != b.S) return a.S > b.S;
    if (a.k.l != b.k.l) return a.k.l < b.k.l;
    if (a.k.k != b.k.k) return a.k.k < b.k.k;
    if (a.k.j != b.k.j) return a.k.j < b.k.j;
    return a.k.i < b.k.i;
  });
  std::vector<Key> journal, stack;
  for (const Cand& c : cand) {
    if (T.state(c.k.l, c.k.i, c.k.j, c.k.k) != Octree::LEAF) continue;
    if (leaves + 7 > max_blocks) {  // any closure adds >= 7 leaves: refused without trying
      res.refused++;
      continue;
    }
    journal.clear();
    stack.assign(1, c.k);
    bool ok = true;
    while (ok && !stack.empty()) {
      const Key n = stack.back();
      stack.pop_back();
      if (T.state(n.l, n.i, n.j, n.k) != Octree::LEAF) continue;
      if (old.state(n.l, n.i, n.j, n.k) != Octree::LEAF) {
        ok = false;  // would refine a leaf created by this remesh
        break;
      }
      T.refine(n.l, n.i, n.j, n.k);
      journal.push_back(n);
      const int lc = n.l + 1;
      for (int ch = 0; ch < 8; ch++) {
        const int ci = 2 * n.i + (ch & 1), cj = 2 * n.j + ((ch >> 1) & 1), ck = 2 * n.k + (ch >> 2);
        for (int q = 0; q < 27; q++) {
          if (q == 13) continue;
          int p[3] = {ci + q % 3 - 1, cj + (q / 3) % 3 - 1, ck + q / 9 - 1};
          bool in = true;
          for (int a = 0; a < 3; a++) in = in && T.wrap(lc, a, p[a]);
          if (!in) continue;
          int lv = lc;
          while (T.state(lv, p[0], p[1], p[2]) == Octree::ABSENT) {
            lv--;
            p[0] >>= 1; p[1] >>= 1; p[2] >>= 1;
          }
          if (lc - lv >= 2) stack.push_back({lv, p[0], p[1], p[2]});
        }
      }
    }
    if (ok && leaves + 7 * int64_t(journal.size()) <= max_blocks) {
      leaves += 7 * int64_t(journal.size());
      res.refined += int64_t(journal.size());
    } else {
      for (auto it = journal.rbegin(); it != journal.rend(); ++it) T.unrefine(it->l, it->i, it->j, it->k);
      res.refused++;
    }
  }
  // coarsening
  std::vector<Key> par;
  for (int64_t s = 0; s < op.nleaf; s++) {
    const Key& k = op.keys[size_t(s)];
    if (k.l == 0 || (k.i & 1) || (k.j & 1) || (k.k & 1)) continue;  // visit each octet once, from its first child
    const Key P{k.l - 1, k.i >> 1, k.j >> 1, k.k >> 1};
    if (T.state(P.l, P.i, P.j, P.k) != Octree::REFINED) continue;
    bool ok = true;
    for (int ch = 0; ch < 8 && ok; ch++) {
      const int ci = 2 * P.i + (ch & 1), cj = 2 * P.j + ((ch >> 1) & 1), ck = 2 * P.k + (ch >> 2);
      const int32_t* it = old_id.find(pk4(P.l + 1, ci, cj, ck));
      if (!it || T.state(P.l + 1, ci, cj, ck) != Octree::LEAF) ok = false;
      else if (!(S[size_t(*it)] < coarsen_slope)) ok = false;
    }
    if (ok) par.push_back(P);
  }
  std::sort(par.begin(), par.end(), [](const Key& a, const Key& b) {
    if (a.l != b.l) return a.l > b.l;
    if (a.k != b.k) return a.k < b.k;
    if (a.j != b.j) return a.j < b.j;
    return a.i < b.i;
  });
  for (const Key& P : par) {
    const int lc = P.l + 1;
    bool ok = true;
    for (int dz = -1; dz <= 2 && ok; dz++)
      for (int dy = -1; dy <= 2 && ok; dy++)
        for (int dx = -1; dx <= 2 && ok; dx++) {
          int p[3] = {2 * P.i + dx, 2 * P.j + dy, 2 * P.k + dz};
          bool in = true;
          for (int a = 0; a < 3; a++) in = in && T.wrap(lc, a, p[a]);
          if (!in) continue;
          if ((p[0] >> 1) == P.i && (p[1] >> 1) == P.j && (p[2] >> 1) == P.k) continue;  // inside P
          if (T.state(lc, p[0], p[1], p[2]) == Octree::REFINED) ok = false;
        }
    if (!ok) continue;
    T.unrefine(P.l, P.i, P.j, P.k);
    res.coarsened++;
  }
  // migration tasks in the new storage order (none when nothing changed:
  // the caller keeps the mesh)
  if (res.refined == 0 && res.coarsened == 0) return res;
  for (const Key& k : T.leaves()) {
    MigrTask t{};
    for (int q = 0; q < 8; q++) t.src[q] = -1;
    const int32_t* it = old_id.find(pk4(k.l, k.i, k.j, k.k));
    const int32_t* par = k.l > 0 ? old_id.find(pk4(k.l - 1, k.i >> 1, k.j >> 1, k.k >> 1)) : nullptr;
    if (it) {
      t.kind = MIGR_COPY;
      t.src[0] = *it;
    } else if (par) {
      t.kind = MIGR_PROLONG;
      t.src[0] = *par;
      t.co = (k.i & 1) | ((k.j & 1) << 1) | ((k.k & 1) << 2);
    } else {
      t.kind = MIGR_RESTRICT;
      for (int ch = 0; ch < 8; ch++) {
        const int32_t* c = old_id.find(pk4(k.l + 1, 2 * k.i + (ch & 1), 2 * k.j + ((ch >> 1) & 1), 2 * k.k + (ch >> 2)));
        if (!c) throw std::logic_error("a merged leaf's children were not all leaves");
        t.src[ch] = *c;
      }
    }
    res.migr.push_back(t);
  }
  return res;
}

}  // namespace amr
