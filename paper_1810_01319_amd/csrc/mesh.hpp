// mesh.hpp -- host side of the array-of-octrees (paper Sec. II-B): octree
// nodes in a hash map, level-by-level 2:1 balance, Morton leaf order, and
// the plan tables the kernels walk.
#pragma once
#include <algorithm>
#include <cstdint>
#include <memory>
#include <string>
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

// Hash table from packed node keys (level << 60 | k << 40 | j << 20 | i; the
// all-ones key never occurs, level <= 8) to small values: open addressing
// with linear probing in one flat array (load <= 1/2, Fibonacci hashing),
// deletion by backward shift.  The plan build and the remesh decisions look
// up every leaf's 26 neighbours; a node-based map made those lookups most of
// the host's remesh time.
template <class V>
class FlatMap {
 public:
  static constexpr uint64_t kEmpty = ~uint64_t(0);
  FlatMap() { rehash(16); }
  size_t size() const { return n_; }
  void clear() {
    std::fill(key_.begin(), key_.end(), kEmpty);
    n_ = 0;
  }
  void reserve(size_t n) {
    size_t c = 16;
    while (c < 2 * n) c <<= 1;
    if (c > key_.size()) rehash(c);
  }
  const V* find(uint64_t k) const {
    for (size_t s = home(k);; s = (s + 1) & mask_) {
      if (key_[s] == k) return &val_[s];
      if (key_[s] == kEmpty) return nullptr;
    }
  }
  V* find(uint64_t k) { return const_cast<V*>(static_cast<const FlatMap*>(this)->find(k)); }
  // The value of k, inserted as V{} if absent.
  V& operator[](uint64_t k) {
    if (2 * (n_ + 1) > key_.size()) rehash(2 * key_.size());
    size_t s = home(k);
    for (; key_[s] != kEmpty; s = (s + 1) & mask_)
      if (key_[s] == k) return val_[s];
    key_[s] = k;
    val_[s] = V{};
    n_++;
    return val_[s];
  }
  void erase(uint64_t k) {
    size_t i = home(k);
    for (; key_[i] != k; i = (i + 1) & mask_)
      if (key_[i] == kEmpty) return;
    // backward shift: move each later entry of the run whose home does not
    // lie cyclically in (i, j] into the hole
    for (size_t j = (i + 1) & mask_; key_[j] != kEmpty; j = (j + 1) & mask_) {
      const size_t h = home(key_[j]);
      const bool stays = i <= j ? (i < h && h <= j) : (i < h || h <= j);
      if (stays) continue;
      key_[i] = key_[j];
      val_[i] = val_[j];
      i = j;
    }
    key_[i] = kEmpty;
    n_--;
  }
  // f(key, value) for every entry, in table order.
  template <class F>
  void for_each(F&& f) const {
    for (size_t s = 0; s < key_.size(); s++)
      if (key_[s] != kEmpty) f(key_[s], val_[s]);
  }

 private:
  size_t home(uint64_t k) const { return size_t((k * 0x9E3779B97F4A7C15ull) >> shift_); }
  void rehash(size_t cap) {
    std::vector<uint64_t> ok = std::move(key_);
    std::vector<V> ov = std::move(val_);
    key_.assign(cap, kEmpty);
    val_.assign(cap, V{});
    mask_ = cap - 1;
    int bits = 0;
    while ((size_t(1) << bits) < cap) bits++;
    shift_ = 64 - bits;
    n_ = 0;
    for (size_t s = 0; s < ok.size(); s++)
      if (ok[s] != kEmpty) (*this)[ok[s]] = ov[s];
  }
  std::vector<uint64_t> key_;
  std::vector<V> val_;
  size_t n_ = 0, mask_ = 0;
  int shift_ = 64;
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
  FlatMap<uint8_t> node_;
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
  // phase-2 tasks: (leaf, neighbour code) pairs whose neighbour position is
  // covered by a coarser leaf, faces first, then edges, then corners
  std::vector<int32_t> p2task;
  // phase-2 waves in leaf order: (task row << kP2SubBits) | wave in task, so
  // that one launch covers a leaf's face, edge and corner regions together
  std::vector<int32_t> p2wave;
  int64_t np2t[3] = {0, 0, 0};   // tasks of each kind (faces, edges, corners)
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
