// Save arrays of in-place streaming on a refined forest.
//
// With the finest level streamed in place, its states at the start of a
// parent step (t) and after the first substep (t + 1/2) are overwritten by
// the next substep, yet the second substep's back-trace and the coarser
// level's coalescence read them: the value f*_a(y) of a cell y whose
// neighbour y + e_a lies in the coarser region, i.e. what y sends into the
// fine ghost layers (section 4).  The in-place launches save exactly those
// values, at t + 1/2 (first substep) and at t + 1 (second substep, for the
// next parent step), in arrays indexed by (slot, direction, face cell).
//
// Layout of one slot: for each direction a = 1 .. 18 one array of n^2 per
// axis along which e_a is nonzero (6 axis directions x 1 + 12 edge
// directions x 2 = 30 arrays).  A value is stored at the face of the first
// axis (x, then y, then z) through which y + e_a leaves the block, indexed
// by y's two other coordinates (u + n v in axis order).
#pragma once

#include <cstdint>

#include "inplace.hpp"
#include "lattice.hpp"

namespace lbm {
namespace dev {

constexpr int kSaveArrays = kSaveArrayCount;

__host__ __device__ constexpr int save_count(int a) { return (ex(a) != 0) + (ey(a) != 0) + (ez(a) != 0); }
// First array of direction a: directions 1 .. 6 lie along one axis, 7 .. 18
// along two (closed form, checked against the sum below), so that a
// direction known only at run time costs no loop.
__host__ __device__ constexpr int save_base(int a) { return a <= 6 ? a - 1 : 6 + 2 * (a - 7); }
constexpr bool save_base_matches() {
  int b = 0;
  for (int d = 1; d < 19; ++d) {
    if (save_base(d) != b) return false;
    b += save_count(d);
  }
  return b == kSaveArrays;
}
static_assert(save_base_matches(), "30 save arrays per slot, axis directions first");

// Components of direction a from packed tables (2 bits per direction,
// component + 1): cheap for a direction known only at run time.
__host__ __device__ constexpr uint64_t pack_components(int axis) {
  uint64_t t = 0;
  for (int a = 0; a < 19; ++a)
    t |= uint64_t((axis == 0 ? ex(a) : axis == 1 ? ey(a) : ez(a)) + 1) << (2 * a);
  return t;
}
template <int AXIS>
__host__ __device__ __forceinline__ int comp_rt(int a) {
  constexpr uint64_t t = pack_components(AXIS);
  return int((t >> (2 * a)) & 3u) - 1;
}

// Index of the value of cell (i, j, k) of block `slot` in direction a, for a
// cell whose neighbour (i, j, k) + e_a lies outside the block.
template <int N>
__device__ __forceinline__ uint64_t save_index(uint32_t slot, int a, int i, int j, int k) {
  const int e[3] = {comp_rt<0>(a), comp_rt<1>(a), comp_rt<2>(a)};
  const int c[3] = {i, j, k};
  int rank = 0, axis = -1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const bool leaves = c[d] + e[d] < 0 || c[d] + e[d] >= N;
    if (axis < 0 && leaves) axis = d;
    if (axis < 0 && e[d] != 0) ++rank;
  }
  if (axis < 0) axis = 0;  // not a leaving value: never asked for; any in-range index
  const int u = axis == 0 ? j : i, v = axis == 2 ? j : k;
  return (uint64_t(slot) * kSaveArrays + uint64_t(save_base(a) + rank)) * uint64_t(N * N) + uint64_t(u + N * v);
}

}  // namespace dev
}  // namespace lbm
