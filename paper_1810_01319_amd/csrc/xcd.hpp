// xcd.hpp -- workgroup renumbering for the 8 XCDs of an MI355X.
//
// Workgroups are dispatched to the XCDs round-robin (workgroup b to XCD
// b mod 8), and each XCD has its own L2.  Renumbered by xcd_block(), each XCD
// takes one contiguous range of the grid's work items, in order, so that work
// items sharing cache lines (neighbouring pencil tiles, the ghost fragments
// of one leaf) meet in the same L2 instead of being fetched from HBM once per
// XCD.  The map is a bijection of [0, gridDim.x): no result depends on it.
#pragma once
#include <hip/hip_runtime.h>

namespace amr {

constexpr unsigned kXcds = 8;

__device__ __forceinline__ unsigned xcd_block() {
  const unsigned G = gridDim.x, b = blockIdx.x;
  const unsigned q = G / kXcds, r = G % kXcds, x = b % kXcds, i = b / kXcds;
  // XCD x < r takes q + 1 items starting at x (q + 1); XCD x >= r takes q
  // items starting at r (q + 1) + (x - r) q
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

}  // namespace amr
