// mesh.hpp -- host side of the array-of-octrees (paper Sec. II-B): octree
// nodes in a hash map, level-by-level 2:1 balance, Morton leaf order, and
// the plan tables the kernels walk.
#pragma once
#include <cstdint>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "layout.hpp"

struct amr_mesh_desc_s;

namespace amr {

struct MeshDesc {
  int32_t root[3];
  int32_t N;
  int32_t max_level;
  int32_t bc[3];
  double gamma, cfl, rho_floor, p_floor;
  int32_t iters;
  int32_t de;  // dual-energy field
  double eta1, eta2;
};

struct Key {
  int32_t l, i, j, k;
};

class Octree {
 public:
  enum : uint8_t { ABSENT = 0, LEAF = 1, REFINED = 2 };

  explicit Octree(const MeshDesc& d);
  const MeshDesc& desc() const { return d_; }

  // Static refinement list; then balance.  Returns "" or an error message.
  std::string refine_list(const int32_t* keys, int64_t n);
  std::string from_leaves(const int32_t* keys, int64_t n);  // validates tiling + balance
  void balance();
  std::string check_balance() const;

  uint8_t state(int l, int i, int j, int k) const;
  int ext(int l, int ax) const { return d_.root[ax] << l; }
  // periodic wrap of a level-l block coordinate; false if outside an
  // outflow boundary
  bool wrap(int l, int ax, int& v) const;
  void refine(int l, int i, int j, int k);
  // undo of refine(): the node becomes a leaf again, its children vanish
  void unrefine(int l, int i, int j, int k);
  // Leaves in storage order: roots x-fastest, Morton (depth-first) inside.
  std::vector<Key> leaves() const;

 private:
  static uint64_t pack(int l, int i, int j, int k) {
    return (uint64_t(l) << 60) | (uint64_t(k) << 40) | (uint64_t(j) << 20) | uint64_t(i);
  }
  void dfs(int l, int i, int j, int k, std::vector<Key>& out) const;
  MeshDesc d_;
  std::unordered_map<uint64_t, uint8_t> node_;
};

// Flattened tables of one or more meshes.
struct Plan {
  int N = 0, M = 0;
  int nf = kFields;  // fields per cell: kFields, or kFieldsDE with the dual-energy field
  int64_t nleaf = 0;
  std::vector<InstParams> inst;
  std::vector<BlockInfo> blocks;
  std::vector<Nbr> nbr;          // 27 per leaf
  std::vector<int32_t> fine;     // 8 per FINE entry
  std::vector<int32_t> p2list;   // leaves with a coarser neighbour
  std::vector<int32_t> faceslot; // 6 per leaf
  std::vector<RefluxTask> reflux[3];
  std::vector<MigrTask> migr;    // set before build() by a remesh
  std::vector<Reloc> reloc;      // per leaf of the previous mesh; set before build() by a remesh
  std::vector<int32_t> reloc_child;  // 8 per split leaf
  int64_t nslots = 0;
  PlanOffsets off{};
  std::vector<unsigned char> staging;  // bytes [0, off.faces) as uploaded
  std::vector<Key> keys;               // per leaf, storage order
  bool has_p2 = false;

  // Build from meshes (all with the same N).  Returns "" or an error.
  std::string build(const std::vector<const Octree*>& meshes);
};

InstParams make_inst_params(const MeshDesc& d);

struct RemeshResult {
  std::unique_ptr<Octree> tree;
  std::vector<MigrTask> migr;  // in the new tree's leaf order
  int64_t refined = 0, coarsened = 0, refused = 0;
};

// Refinement decisions of a remesh from the per-leaf indicator S (in the
// old plan's leaf order); see the reading in mesh.cpp.
RemeshResult remesh_decide(const Octree& old, const Plan& old_plan, const std::vector<double>& S,
                           double refine_slope, double coarsen_slope, int64_t max_blocks);

}  // namespace amr
