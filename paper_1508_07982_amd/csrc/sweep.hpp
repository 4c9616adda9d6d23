// The fused refined-LBM sweep kernel for gfx950 (templates; instantiated per
// storage form in sweep_f64.hip, sweep_f32.hip and sweep_f16.hip).
//
// One launch of `sweep_kernel` performs one substep of one level L
// (section 4, Algorithm 1, in post-collision form).  Its work list holds the
// level-L blocks only; nothing is stored or computed for ghost cells.  For
// every interior cell x of level L and every direction a the pulled value is
//   - (x, a) in the coalescence set (x - e_a, or for an edge direction one
//     of its axis projections, lies in region(L+1)) -> the mean of the 8
//     children of x after the finer level's two substeps (eq. ftoc), computed
//     before this sweep by the coalescence (coalesce.hpp: a launch of its own,
//     or workgroups of the finer level's second-substep launch);
//   - source x - e_a inside a level-L block -> that block's value;
//   - source in the coarser region (a virtual level-L cell of a ghost
//     layer), reconstructed by a back-trace instead of a stored halo:
//         substep 1: the parent's post-collision value (explosion eq. ctof,
//                    done as a gather);
//         substep 2: the value that the first substep streamed into the
//                    ghost cell x - e_a, i.e. the level's own state at t at
//                    x - 2 e_a if that is a level-L cell, else the parent's
//                    value (ghost layers stream, never collide).
// Every interior cell is then collided (SRT, eq. fequ; or TRT with a body
// force) and written.
//
// The stored state is post-collision: the collision that Algorithm 1 does at
// the start of the next step is done at the end of this one.  Moments and
// the coarse-to-fine values read by the finer level are unaffected, since
// collision conserves rho and u and the finer level reads the coarse
// post-collision state in both forms.
//
// PDFs are stored shifted, h = f - w (FP64, FP32 or FP16); arithmetic is in
// the shifted form: drho = sum h, u = sum e h, h_eq = w (drho + 3 e.u +
// 4.5 (e.u)^2 - 1.5 u^2), h <- h + omega (h_eq - h).
//
// Memory layout per level: [slot][direction][z][y][x] (block-major, one
// slot per block), so a 64-lane wavefront reads 64 consecutive cells of one
// direction and the 19 rows of a tile lie inside one block's storage.
#pragma once

#include "coalesce.hpp"
#include "forest.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

namespace lbm {
namespace dev {

// The slot's neighbour table and, for a slot with finer neighbours, its row
// in the coalesced-value buffers.  Every lane of a workgroup sweeps the same
// slot, so the table is loaded once per lane into scalar registers (no LDS
// copy and no barrier before the first PDF load) and indexed only with
// compile-time offsets (see pick).
struct SlotCache {
  int32_t nbr[27];
  int32_t fine_row;
};

template <int X, int Y, int Z>
__device__ __forceinline__ int32_t nbr_at(const SlotCache& sc) {
  return sc.nbr[13 + X + 3 * Y + 9 * Z];
}
template <int DX, int Y, int Z>
__device__ __forceinline__ int32_t pick_x(const SlotCache& sc, bool bx) {
  if constexpr (DX == 0)
    return nbr_at<0, Y, Z>(sc);
  else
    return bx ? nbr_at<DX, Y, Z>(sc) : nbr_at<0, Y, Z>(sc);
}
template <int DX, int DY, int Z>
__device__ __forceinline__ int32_t pick_xy(const SlotCache& sc, bool bx, bool by) {
  if constexpr (DY == 0)
    return pick_x<DX, 0, Z>(sc, bx);
  else
    return by ? pick_x<DX, DY, Z>(sc, bx) : pick_x<DX, 0, Z>(sc, bx);
}
// Table entry of the neighbour offset whose components are DX, DY, DZ
// where bx, by, bz are set and 0 elsewhere.  A shift by -e_a (or -2 e_a)
// leaves the block only through the faces the direction points away from,
// so every lookup of direction a has this form with (DX, DY, DZ) = -e_a:
// at most 8 candidates, selected per lane from the scalar table.
template <int DX, int DY, int DZ>
__device__ __forceinline__ int32_t pick(const SlotCache& sc, bool bx, bool by, bool bz) {
  if constexpr (DZ == 0)
    return pick_xy<DX, DY, 0>(sc, bx, by);
  else
    return bz ? pick_xy<DX, DY, DZ>(sc, bx, by) : pick_xy<DX, DY, 0>(sc, bx, by);
}

// Whether a local coordinate lies outside [0, N).
template <int N>
__device__ __forceinline__ bool outside(int c) {
  return c < 0 || c >= N;
}

// Neighbour offset (-1, 0, +1) of a local coordinate after a shift.
template <int N>
__device__ __forceinline__ int side(int c) {
  return c < 0 ? -1 : (c >= N ? 1 : 0);
}

// Address of level-L cell (lx, ly, lz) of the virtual block whose neighbour
// table entry is `code` (< kNbrFine, i.e. inside a level-(L-1) leaf): the
// parent's post-collision value (homogeneous explosion, eq. ctof).  A parent
// cell on the parent block's x face through which direction A leaves it is
// read from the parent's x-face copy: across an x-face interface all the
// parents lie there, one per 128-byte line in the block-major buffer and
// contiguous in the copy.
template <typename S, int N, int A>
__device__ __forceinline__ const S* parent_ptr(const SweepArgs& a, int code, int lx, int ly, int lz) {
  constexpr int H = Geo<S, N>::H;
  const int pp = kNbrCoarse0 - code;
  const int oc = pp & 7;
  const int px = (oc & 1 ? H : 0) + (lx >> 1), py = (oc & 2 ? H : 0) + (ly >> 1), pz = (oc & 4 ? H : 0) + (lz >> 1);
  if constexpr (ex(A) != 0) {
    if (px == (ex(A) > 0 ? N - 1 : 0))
      return static_cast<const S*>(a.par_face) + xface_index<S, N, A>(uint32_t(pp >> 3), uint32_t(py + N * pz));
  }
  return static_cast<const S*>(a.par) + pdf_index<N>(A, uint32_t(pp >> 3), uint32_t(px + N * (py + N * pz)));
}

// Special sources of cell x = (i, j, k) of block `slot`, direction A.
//
// No-slip wall (x - e_A lies beyond a non-periodic end, section 2.2): the
// boundary cell holds what x sent towards it, reversed -- x's own value of
// the opposite direction in the state being streamed (halfway bounce-back).
// Coarse source (the cell x - e_A lies in a level-(L-1) leaf):
//   substep 1: the exploded parent value of x - e_A;
//   substep 2: x - e_A is a halo cell whose first-substep value was pulled
//   from x - 2 e_A: the level's own state at t there, the exploded parent
//   value if x - 2 e_A is also in the coarse region, or, if x - 2 e_A is a
//   wall, the halo cell's own bounced-back value: its exploded parent value
//   of the opposite direction (ghost layers get the boundary treatment too,
//   section 4.1).
// coarse_source returns its address (an inconsistent table sets an error
// bit and yields an in-bounds dummy address), so that the loads of all
// cells of a lane can be issued together.
template <typename S, int N, int A>
__device__ __forceinline__ const S* coarse_source(const SweepArgs& a, const SlotCache& sc, int slot, int i, int j,
                                                  int k) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const S* dummy = static_cast<const S*>(a.cur);
  const int sx = i - EX, sy = j - EY, sz = k - EZ;
  const int code = pick<-EX, -EY, -EZ>(sc, outside<N>(sx), outside<N>(sy), outside<N>(sz));
  if (code == kNbrWall) return static_cast<const S*>(a.cur) + pdf_index<N>(opp(A), uint32_t(slot), uint32_t(i + N * (j + N * k)));
  if (code > kNbrCoarse0) {  // not a coarse region: never expected here
    atomicOr(a.err, kErrNoSource);
    return dummy;
  }
  if (a.substep == 1) return parent_ptr<S, N, A>(a, code, sx & (N - 1), sy & (N - 1), sz & (N - 1));
  const int zx = sx - EX, zy = sy - EY, zz = sz - EZ;
  const int cz = pick<-EX, -EY, -EZ>(sc, outside<N>(zx), outside<N>(zy), outside<N>(zz));
  if (cz >= 0)
    return static_cast<const S*>(a.prev) +
           pdf_index<N>(A, uint32_t(cz), uint32_t((zx & (N - 1)) + N * ((zy & (N - 1)) + N * (zz & (N - 1)))));
  if (cz == kNbrWall) return parent_ptr<S, N, opp(A)>(a, code, sx & (N - 1), sy & (N - 1), sz & (N - 1));
  if (cz > kNbrCoarse0) {
    atomicOr(a.err, kErrNoSource);
    return dummy;
  }
  return parent_ptr<S, N, A>(a, cz, zx & (N - 1), zy & (N - 1), zz & (N - 1));
}

// The same special sources as a value, with the interpolated explosion:
// every exploded parent value becomes the reconstruction at the fine cell
// (interp_value in lattice.hpp, with the parents' level table).  Only the
// sweep variant for the interpolated explosion calls it, for the cells of a
// lane whose source is special; the direction is a run-time argument and the
// function is not inlined, which keeps that variant small.  code and cz are
// the block's table entries of x - e_A and x - 2 e_A, which the caller holds
// in registers.
template <typename S, int N>
__device__ __noinline__ typename Form<S>::C coarse_value_rt(const S* cur, const S* prev, const S* par,
                                                            const int32_t* par_nbr, int* err, int substep, int slot,
                                                            int A, int i, int j, int k, int code, int cz) {
  using C = typename Form<S>::C;
  constexpr int H = Geo<S, N>::H;
  const int EX = ex(A), EY = ey(A), EZ = ez(A);
  auto parent = [&](int code, int lx, int ly, int lz, int aa) -> C {
    const int pp = kNbrCoarse0 - code;
    const int oc = pp & 7, pslot = pp >> 3;
    return interp_value<S, N>(par, par_nbr + int64_t(pslot) * 27, (oc & 1 ? H : 0) + (lx >> 1),
                              (oc & 2 ? H : 0) + (ly >> 1), (oc & 4 ? H : 0) + (lz >> 1), aa, lx & 1, ly & 1, lz & 1,
                              err);
  };
  const int sx = i - EX, sy = j - EY, sz = k - EZ;
  if (code == kNbrWall) return Form<S>::ld(cur + pdf_index<N>(opp(A), uint32_t(slot), uint32_t(i + N * (j + N * k))));
  if (code > kNbrCoarse0) {
    atomicOr(err, kErrNoSource);
    return C(0);
  }
  if (substep == 1) return parent(code, sx & (N - 1), sy & (N - 1), sz & (N - 1), A);
  const int zx = sx - EX, zy = sy - EY, zz = sz - EZ;
  if (cz >= 0)
    return Form<S>::ld(prev + pdf_index<N>(A, uint32_t(cz), uint32_t((zx & (N - 1)) + N * ((zy & (N - 1)) + N * (zz & (N - 1))))));
  if (cz == kNbrWall) return parent(code, sx & (N - 1), sy & (N - 1), sz & (N - 1), opp(A));
  if (cz > kNbrCoarse0) {
    atomicOr(err, kErrNoSource);
    return C(0);
  }
  return parent(cz, zx & (N - 1), zy & (N - 1), zz & (N - 1), A);
}

template <typename S, int N, int A>
__device__ __forceinline__ typename Form<S>::C coarse_value(const SweepArgs& a, const SlotCache& sc, int slot, int i, int j,
                                                           int k) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const int sx = i - EX, sy = j - EY, sz = k - EZ;
  const int code = pick<-EX, -EY, -EZ>(sc, outside<N>(sx), outside<N>(sy), outside<N>(sz));
  const int cz = pick<-EX, -EY, -EZ>(sc, outside<N>(sx - EX), outside<N>(sy - EY), outside<N>(sz - EZ));
  return coarse_value_rt<S, N>(static_cast<const S*>(a.cur), static_cast<const S*>(a.prev),
                               static_cast<const S*>(a.par), a.par_nbr, a.err, a.substep, slot, A, i, j, k, code, cz);
}

// Coalescence (eq. ftoc): the value of a coalesced pair comes from the
// coalescence launch that precedes this sweep (see CoalArgs), stored like
// the state at the slot's fine row, or in the x-face layout for a pair that
// enters through an x face.
template <typename S, int N, int A>
__device__ __forceinline__ const S* coalesced_source(const SweepArgs& a, const SlotCache& sc, int i, int j, int k) {
  constexpr int EX = ex(A);
  if constexpr (EX != 0) {
    if (i == (EX == 1 ? 0 : N - 1))
      return static_cast<const S*>(a.coal_x) + xface_index<S, N, A>(uint32_t(sc.fine_row), uint32_t(j + N * k));
  }
  return static_cast<const S*>(a.coal) + pdf_index<N>(A, uint32_t(sc.fine_row), uint32_t(i + N * (j + N * k)));
}

// Ordinary pull of direction A for the W cells (i0 .. i0+W-1, j, k) of one
// lane, in two phases so that every load of the lane is in flight before
// the first one is used:
//   issue_dir: one vector load of the source row into h[A] and, for
//              x-shifted directions, one element load into edge[] from the
//              x neighbour's x-face copy (every lane of a row loads the
//              row end's element, so no branch and no wait splits the
//              loads and the row's lanes share one address);
//   shift_dir: the x shift of the row by one cell, a DPP move between
//              lanes, with the edge element at the end of the row.
// A source block that is not a level-L block sets `odd` (the address is
// then replaced by the lane's own, so every load stays inside the buffer).
template <typename S, int N, int A, bool SIMPLE>
__device__ __forceinline__ void issue_dir(const SweepArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                          typename Form<S>::C (*h)[Geo<S, N>::W], typename Form<S>::C* edge,
                                          uint32_t& odd) {
  constexpr int W = Geo<S, N>::W;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const int sy = j - EY, sz = k - EZ;
  const bool by = outside<N>(sy), bz = outside<N>(sz);
  const uint32_t row = uint32_t(N * ((sy & (N - 1)) + N * (sz & (N - 1))));
  const int nbm = pick<0, -EY, -EZ>(sc, false, by, bz);
  if (!SIMPLE) odd |= uint32_t(nbm < 0);
  const S* __restrict__ base = static_cast<const S*>(a.cur);
  const uint64_t bm = pdf_index<N>(A, uint32_t(SIMPLE || nbm >= 0 ? nbm : slot), row + uint32_t(i0));
  Vec<S>::load(base + bm, h[A]);
  if constexpr (EX != 0) {
    const bool at_end = EX == 1 ? i0 == 0 : i0 == N - W;
    const int nbx = pick<-EX, -EY, -EZ>(sc, true, by, bz);
    if (!SIMPLE) odd |= uint32_t(at_end && nbx < 0);
    // the end element of the x neighbour's source row, cell N - 1 (EX = 1)
    // or 0 (EX = -1): a value leaving that block through its x face
    const int eb = SIMPLE || nbx >= 0 ? nbx : slot;
    edge[xdir_index(A)] = Form<S>::ld(static_cast<const S*>(a.face_cur) + xface_index<S, N, A>(uint32_t(eb), row / N));
  }
}

template <typename S, int N, int A>
__device__ __forceinline__ void shift_dir(int i0, typename Form<S>::C (*h)[Geo<S, N>::W],
                                          const typename Form<S>::C* edge) {
  using C = typename Form<S>::C;
  constexpr int W = Geo<S, N>::W;
  constexpr int EX = ex(A);
  if constexpr (EX == 1) {  // source x - 1
    const C prev = dpp_move<kDppRowShr1>(h[A][W - 1]);
#pragma unroll
    for (int c = W - 1; c > 0; --c) h[A][c] = h[A][c - 1];
    h[A][0] = i0 == 0 ? edge[xdir_index(A)] : prev;
  } else if constexpr (EX == -1) {  // source x + 1
    const C next = dpp_move<kDppRowShl1>(h[A][0]);
#pragma unroll
    for (int c = 0; c < W - 1; ++c) h[A][c] = h[A][c + 1];
    h[A][W - 1] = i0 == N - W ? edge[xdir_index(A)] : next;
  }
}

template <typename S, int N, bool SIMPLE, int A = 0>
__device__ __forceinline__ void issue_all(const SweepArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                          typename Form<S>::C (*h)[Geo<S, N>::W], typename Form<S>::C* edge,
                                          uint32_t& odd) {
  issue_dir<S, N, A, SIMPLE>(a, sc, slot, i0, j, k, h, edge, odd);
  if constexpr (A + 1 < 19) issue_all<S, N, SIMPLE, A + 1>(a, sc, slot, i0, j, k, h, edge, odd);
}

template <typename S, int N, int A = 0>
__device__ __forceinline__ void shift_all(int i0, typename Form<S>::C (*h)[Geo<S, N>::W],
                                          const typename Form<S>::C* edge) {
  shift_dir<S, N, A>(i0, h, edge);
  if constexpr (A + 1 < 19) shift_all<S, N, A + 1>(i0, h, edge);
}

template <typename S, int N, bool SIMPLE>
__device__ __forceinline__ void pull_all(const SweepArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                         typename Form<S>::C (*h)[Geo<S, N>::W], uint32_t& odd) {
  typename Form<S>::C edge[kXDirs];
  issue_all<S, N, SIMPLE>(a, sc, slot, i0, j, k, h, edge, odd);
  shift_all<S, N>(i0, h, edge);
}

// The slot's neighbour table as two 27-bit masks: neighbours that are not
// level-L blocks (bit d for table entry d < 0) and finer neighbours
// (entry d == kNbrFine), computed from the scalar table; the per-direction
// tests below are then bit tests.
struct NbrMasks {
  uint32_t other;
  uint32_t fine;
};
__device__ __forceinline__ NbrMasks nbr_masks(const SlotCache& sc) {
  NbrMasks m{0u, 0u};
#pragma unroll
  for (int d = 0; d < 27; ++d) {
    const int32_t v = sc.nbr[d];
    m.other |= uint32_t(v < 0) << d;
    m.fine |= uint32_t(v == kNbrFine) << d;
  }
  // the table is the workgroup's: make the masks wave-uniform (scalar)
  m.other = uint32_t(__builtin_amdgcn_readfirstlane(int(m.other)));
  m.fine = uint32_t(__builtin_amdgcn_readfirstlane(int(m.fine)));
  return m;
}

// Cells of a lane whose direction-A source is not an ordinary level-L read:
// bit c of the returned mask; bit c of `co` marks a coalesced pair, i.e.
// x - e_A or (edge directions) one of its axis projections in region(L+1).
template <int N, int W, int A>
__device__ __forceinline__ uint32_t special_cells(NbrMasks m, uint32_t fl, int i0, int j, int k, uint32_t& co) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  // keep each direction's tests next to its use (an empty asm on the scalar
  // masks stops the compiler from evaluating all 19 directions up front)
  asm volatile("" : "+s"(m.other), "+s"(m.fine));
  const int oy = EY == 0 ? 0 : side<N>(j - EY);
  const int oz = EZ == 0 ? 0 : side<N>(k - EZ);
  uint32_t spec = 0;
  co = 0;
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int ox = EX == 0 ? 0 : side<N>(i0 + c - EX);
    const int d = 13 + ox + 3 * oy + 9 * oz;
    uint32_t coal = 0;
    if (fl & kHasFine) {
      coal = (m.fine >> d) & 1u;
      if (A >= 7) {
        const int dA = EX != 0 ? 13 + ox : 13 + 3 * oy;
        const int dB = EZ != 0 ? 13 + 9 * oz : 13 + 3 * oy;
        coal |= ((m.fine >> dA) | (m.fine >> dB)) & 1u;
      }
    }
    spec |= (coal | ((m.other >> d) & 1u)) << c;
    co |= coal << c;
  }
  return spec;
}

// Special sources of direction A for the W cells of a lane (coarse sources
// and coalesced pairs), addressed first and loaded together: one memory
// round trip per direction.
template <typename S, int N, bool INTERP, int A = 0>
__device__ __forceinline__ void fixups(const SweepArgs& a, const SlotCache& sc, int slot, const NbrMasks& m, uint32_t fl, int i0,
                                       int j, int k, typename Form<S>::C (*h)[Geo<S, N>::W]) {
  using C = typename Form<S>::C;
  constexpr int W = Geo<S, N>::W;
  uint32_t co;
  const uint32_t spec = special_cells<N, W, A>(m, fl, i0, j, k, co);
  if (INTERP && spec) {
#pragma unroll
    for (int c = 0; c < W; ++c)
      if ((spec >> c) & 1u)
        h[A][c] = (co >> c) & 1u ? C(Form<S>::ld(coalesced_source<S, N, A>(a, sc, i0 + c, j, k)))
                                 : coarse_value<S, N, A>(a, sc, slot, i0 + c, j, k);
  } else if (spec) {
    C v[W];
#pragma unroll
    for (int c = 0; c < W; ++c) {
      const S* p = !((spec >> c) & 1u) ? static_cast<const S*>(a.cur)
                   : (co >> c) & 1u    ? coalesced_source<S, N, A>(a, sc, i0 + c, j, k)
                                       : coarse_source<S, N, A>(a, sc, slot, i0 + c, j, k);
      v[c] = Form<S>::ld(p);
    }
#pragma unroll
    for (int c = 0; c < W; ++c)
      if ((spec >> c) & 1u) h[A][c] = v[c];
  }
  if constexpr (A + 1 < 19) fixups<S, N, INTERP, A + 1>(a, sc, slot, m, fl, i0, j, k, h);
}

// Relaxation of the opposite pair (A, A + 1), e_{A+1} = -e_A: with
// t = e_A . u the two equilibria share the even part w (drho - 1.5 u^2 +
// 4.5 t^2) and differ in the sign of the odd part 3 w t, and
// h + omega (h_eq - h) = (1 - omega) h + omega h_eq.
template <typename C, int W, int A = 1>
__device__ __forceinline__ void relax_pairs(C (*h)[W], int c, C base, C ux, C uy, C uz, C omc, C ow1, C ow2) {
#pragma clang fp contract(on)
  const C ow = wgt<C>(A) == wgt<C>(1) ? ow1 : ow2;  // omega w_A
  C t = C(0);
  if constexpr (ex(A) != 0) t += ex(A) > 0 ? ux : -ux;
  if constexpr (ey(A) != 0) t += ey(A) > 0 ? uy : -uy;
  if constexpr (ez(A) != 0) t += ez(A) > 0 ? uz : -uz;
  const C even = ow * (base + C(4.5) * t * t);
  const C odd = (C(3) * ow) * t;
  h[A][c] = omc * h[A][c] + (even + odd);
  h[A + 1][c] = omc * h[A + 1][c] + (even - odd);
  if constexpr (A + 2 < 19) relax_pairs<C, W, A + 2>(h, c, base, ux, uy, uz, omc, ow1, ow2);
}

// SRT collision of cell c in shifted form (rho0 = 1).  Multiply-adds are
// fused only within one expression (contract(on)), so every kernel that
// inlines the collision rounds it the same way: the in-place and the
// two-buffer streaming give bitwise equal results.
template <typename C, int W>
__device__ __forceinline__ void collide(C (*h)[W], int c, C om) {
#pragma clang fp contract(on)
  C drho = h[0][c], ux = C(0), uy = C(0), uz = C(0);
#pragma unroll
  for (int a = 1; a < 19; a += 2) {  // opposite pairs (a, a + 1)
    drho += h[a][c] + h[a + 1][c];
    const C d = h[a][c] - h[a + 1][c];
    if (ex(a)) ux += ex(a) > 0 ? d : -d;
    if (ey(a)) uy += ey(a) > 0 ? d : -d;
    if (ez(a)) uz += ez(a) > 0 ? d : -d;
  }
  const C base = drho - C(1.5) * (ux * ux + uy * uy + uz * uz);
  const C omc = C(1) - om;
  h[0][c] = omc * h[0][c] + (om * wgt<C>(0)) * base;
  relax_pairs<C, W>(h, c, base, ux, uy, uz, omc, om * wgt<C>(1), om * wgt<C>(7));
}

// x-face copy of the lane's output (see CoalArgs): the lanes at the two ends
// of a row also write the values of their end cell that leave the block
// through the x face there (directions with e_x = SIDE).
template <typename S, int N, int SIDE, int A = 1>
__device__ __forceinline__ void store_face_side(S* __restrict__ f, uint64_t row, uint32_t jk,
                                                typename Form<S>::C (*h)[Geo<S, N>::W]) {
  if constexpr (ex(A) == SIDE) Form<S>::st(f + xface_index<S, N, A>(row, jk), h[A][SIDE < 0 ? 0 : Geo<S, N>::W - 1]);
  if constexpr (A + 1 < 19) store_face_side<S, N, SIDE, A + 1>(f, row, jk, h);
}
template <typename S, int N>
__device__ __forceinline__ void store_faces(const SweepArgs& a, int row, int i0, int j, int k,
                                            typename Form<S>::C (*h)[Geo<S, N>::W]) {
  S* __restrict__ f = static_cast<S*>(a.face_out);
  const uint32_t jk = uint32_t(j + N * k);
  if (i0 == 0) store_face_side<S, N, -1>(f, uint64_t(row), jk, h);
  if (i0 == N - Geo<S, N>::W) store_face_side<S, N, 1>(f, uint64_t(row), jk, h);
}

// TRT collision with a constant body force (section 2, TRT model and
// external forces) of cell c, in shifted form.  For the opposite pair
// (A, A + 1) the even and odd parts of h - h_eq relax with lambda_e and
// lambda_o, h_eq+ = w (drho - 1.5 u^2 + 4.5 t^2), h_eq- = 3 w t with
// t = e_A . u, and F_A = 3 w_A e_A . a is added (F_{A+1} = -F_A):
//   h_A     <- h_A     - lambda_e (h+ - h_eq+) - [lambda_o (h- - h_eq-) - F_A]
//   h_{A+1} <- h_{A+1} - lambda_e (h+ - h_eq+) + [lambda_o (h- - h_eq-) - F_A].
// u in h_eq is the unmodified sum e h.
template <typename C, int W, int A = 1>
__device__ __forceinline__ void relax_pairs_trt(C (*h)[W], int c, C base, C ux, C uy, C uz, C le, C lo, C ax, C ay,
                                                C az) {
#pragma clang fp contract(on)
  const C w = wgt<C>(A);
  C t = C(0), ta = C(0);
  if constexpr (ex(A) != 0) t += ex(A) > 0 ? ux : -ux, ta += ex(A) > 0 ? ax : -ax;
  if constexpr (ey(A) != 0) t += ey(A) > 0 ? uy : -uy, ta += ey(A) > 0 ? ay : -ay;
  if constexpr (ez(A) != 0) t += ez(A) > 0 ? uz : -uz, ta += ez(A) > 0 ? az : -az;
  const C hp = C(0.5) * (h[A][c] + h[A + 1][c]);
  const C hm = C(0.5) * (h[A][c] - h[A + 1][c]);
  const C dp = le * (hp - w * (base + C(4.5) * t * t));
  const C dm = lo * (hm - C(3) * w * t) - C(3) * w * ta;
  h[A][c] = h[A][c] - dp - dm;
  h[A + 1][c] = h[A + 1][c] - dp + dm;
  if constexpr (A + 2 < 19) relax_pairs_trt<C, W, A + 2>(h, c, base, ux, uy, uz, le, lo, ax, ay, az);
}
template <typename C, int W>
__device__ __forceinline__ void collide_trt(C (*h)[W], int c, C le, C lo, C ax, C ay, C az) {
#pragma clang fp contract(on)
  C drho = h[0][c], ux = C(0), uy = C(0), uz = C(0);
#pragma unroll
  for (int a = 1; a < 19; a += 2) {
    drho += h[a][c] + h[a + 1][c];
    const C d = h[a][c] - h[a + 1][c];
    if (ex(a)) ux += ex(a) > 0 ? d : -d;
    if (ey(a)) uy += ey(a) > 0 ? d : -d;
    if (ez(a)) uz += ez(a) > 0 ? d : -d;
  }
  const C base = drho - C(1.5) * (ux * ux + uy * uy + uz * uz);
  h[0][c] = h[0][c] - le * (h[0][c] - wgt<C>(0) * base);
  relax_pairs_trt<C, W>(h, c, base, ux, uy, uz, le, lo, ax, ay, az);
}

// The collision of cell c: SRT, or TRT with the body force.
template <typename S, bool TRT, typename C, int W>
__device__ __forceinline__ void collide_cell(const SweepArgs& a, C (*h)[W], int c) {
  if constexpr (TRT)
    collide_trt<C, W>(h, c, C(Form<S>::omega(a)), C(Form<S>::lambda_o(a)), C(Form<S>::accel(a, 0)),
                      C(Form<S>::accel(a, 1)), C(Form<S>::accel(a, 2)));
  else
    collide<C, W>(h, c, C(Form<S>::omega(a)));
}

template <typename S, int N, bool SIMPLE, bool TRT, bool INTERP>
__device__ __forceinline__ void update_lane(const SweepArgs& a, const SlotCache& sc, int slot, uint32_t fl, int cell0) {
  using C = typename Form<S>::C;
  constexpr int W = Geo<S, N>::W, N3 = Geo<S, N>::N3;
  const int i0 = cell0 & (N - 1), j = (cell0 / N) & (N - 1), k = cell0 / (N * N);
  C h[19][W];
  uint32_t odd = 0;
  pull_all<S, N, SIMPLE>(a, sc, slot, i0, j, k, h, odd);
  if (!SIMPLE && odd) fixups<S, N, INTERP>(a, sc, slot, nbr_masks(sc), fl, i0, j, k, h);
  if (a.collide) {
#pragma unroll
    for (int c = 0; c < W; ++c) collide_cell<S, TRT>(a, h, c);
  }
  S* __restrict__ nxt = static_cast<S*>(a.nxt) + pdf_index<N>(0, uint32_t(slot), uint32_t(cell0));
#pragma unroll
  for (int d = 0; d < 19; ++d) Vec<S>::store(nxt + d * N3, h[d]);
  if (a.face_out) store_faces<S, N>(a, slot, i0, j, k, h);
}

// ---- packed FP16 path: 8 cells per lane as 4 registers of half pairs ------
//
// Register q of direction A holds cells 2q (low half) and 2q + 1 (high
// half) of the lane's row segment.  The x shift by one cell is a funnel
// shift of neighbouring pairs by 16 bits (the pair across the lane
// boundary comes from a DPP move or from the edge element), so the pulled
// values stay packed; each pair is unpacked to FP32 only for its collision.
// Special sources (coalescence, explosion) are evaluated in FP32 and
// stored into the packed row rounded to FP16, as a ghost layer in FP16
// storage would hold them.
__device__ __forceinline__ float half_lo(uint32_t q) { return __half2float(__ushort_as_half(uint16_t(q & 0xFFFFu))); }
__device__ __forceinline__ float half_hi(uint32_t q) { return __half2float(__ushort_as_half(uint16_t(q >> 16))); }
__device__ __forceinline__ uint32_t half_bits(float v) { return uint32_t(__half_as_ushort(__float2half_rn(keep_fp32(v)))); }
__device__ __forceinline__ uint32_t pack_pair(float lo, float hi) { return half_bits(lo) | (half_bits(hi) << 16); }
// (hi:lo) >> 16: the high half of lo and the low half of hi
__device__ __forceinline__ uint32_t funnel16(uint32_t hi, uint32_t lo) { return __builtin_amdgcn_alignbit(hi, lo, 16); }
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_move_u32(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, 0xF, 0xF, true));
}

template <int N, int A, bool SIMPLE>
__device__ __forceinline__ void issue_dir_h8(const SweepArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                             uint32_t (*q)[4], uint32_t* edge, uint32_t& odd) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const int sy = j - EY, sz = k - EZ;
  const bool by = outside<N>(sy), bz = outside<N>(sz);
  const uint32_t row = uint32_t(N * ((sy & (N - 1)) + N * (sz & (N - 1))));
  const int nbm = pick<0, -EY, -EZ>(sc, false, by, bz);
  if (!SIMPLE) odd |= uint32_t(nbm < 0);
  const uint16_t* __restrict__ base = static_cast<const uint16_t*>(a.cur);
  const int bms = SIMPLE || nbm >= 0 ? nbm : slot;
  const uint4 v = *reinterpret_cast<const uint4*>(base + pdf_index<N>(A, uint32_t(bms), row + uint32_t(i0)));
  q[A][0] = v.x, q[A][1] = v.y, q[A][2] = v.z, q[A][3] = v.w;
  if constexpr (EX != 0) {
    const bool at_end = EX == 1 ? i0 == 0 : i0 == N - 8;
    const int nbx = pick<-EX, -EY, -EZ>(sc, true, by, bz);
    if (!SIMPLE) odd |= uint32_t(at_end && nbx < 0);
    const int eb = SIMPLE || nbx >= 0 ? nbx : slot;  // as in issue_dir
    edge[xdir_index(A)] = static_cast<const uint16_t*>(a.face_cur)[xface_index<__half, N, A>(uint32_t(eb), row / N)];
  }
}

template <int N, int A>
__device__ __forceinline__ void shift_dir_h8(int i0, uint32_t (*q)[4], const uint32_t* edge) {
  constexpr int EX = ex(A);
  if constexpr (EX == 1) {  // cell c takes cell c - 1
    const uint32_t prev = dpp_move_u32<kDppRowShr1>(q[A][3]);
    const uint32_t in = i0 == 0 ? edge[xdir_index(A)] << 16 : prev;
    q[A][3] = funnel16(q[A][3], q[A][2]);
    q[A][2] = funnel16(q[A][2], q[A][1]);
    q[A][1] = funnel16(q[A][1], q[A][0]);
    q[A][0] = funnel16(q[A][0], in);
  } else if constexpr (EX == -1) {  // cell c takes cell c + 1
    const uint32_t next = dpp_move_u32<kDppRowShl1>(q[A][0]);
    const uint32_t in = i0 == N - 8 ? edge[xdir_index(A)] : next;
    q[A][0] = funnel16(q[A][1], q[A][0]);
    q[A][1] = funnel16(q[A][2], q[A][1]);
    q[A][2] = funnel16(q[A][3], q[A][2]);
    q[A][3] = funnel16(in, q[A][3]);
  }
}

template <int N, bool SIMPLE, int A = 0>
__device__ __forceinline__ void issue_all_h8(const SweepArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                             uint32_t (*q)[4], uint32_t* edge, uint32_t& odd) {
  issue_dir_h8<N, A, SIMPLE>(a, sc, slot, i0, j, k, q, edge, odd);
  if constexpr (A + 1 < 19) issue_all_h8<N, SIMPLE, A + 1>(a, sc, slot, i0, j, k, q, edge, odd);
}

template <int N, int A = 0>
__device__ __forceinline__ void shift_all_h8(int i0, uint32_t (*q)[4], const uint32_t* edge) {
  shift_dir_h8<N, A>(i0, q, edge);
  if constexpr (A + 1 < 19) shift_all_h8<N, A + 1>(i0, q, edge);
}

__device__ __forceinline__ void set_half(uint32_t& w, int hi, float v) {
  w = hi ? ((w & 0xFFFFu) | (half_bits(v) << 16)) : ((w & 0xFFFF0000u) | half_bits(v));
}

template <int N, bool INTERP, int A = 0>
__device__ __forceinline__ void fixups_h8(const SweepArgs& a, const SlotCache& sc, int slot, const NbrMasks& m, uint32_t fl,
                                          int i0, int j, int k, uint32_t (*q)[4]) {
  uint32_t co;
  const uint32_t spec = special_cells<N, 8, A>(m, fl, i0, j, k, co);
  if (INTERP && spec) {
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if ((spec >> c) & 1u)
        set_half(q[A][c >> 1], c & 1,
                 (co >> c) & 1u ? Form<__half>::ld(coalesced_source<__half, N, A>(a, sc, i0 + c, j, k))
                                : coarse_value<__half, N, A>(a, sc, slot, i0 + c, j, k));
  } else if (spec) {
    float v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const __half* p = !((spec >> c) & 1u) ? static_cast<const __half*>(a.cur)
                        : (co >> c) & 1u    ? coalesced_source<__half, N, A>(a, sc, i0 + c, j, k)
                                            : coarse_source<__half, N, A>(a, sc, slot, i0 + c, j, k);
      v[c] = Form<__half>::ld(p);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if ((spec >> c) & 1u) set_half(q[A][c >> 1], c & 1, v[c]);
  }
  if constexpr (A + 1 < 19) fixups_h8<N, INTERP, A + 1>(a, sc, slot, m, fl, i0, j, k, q);
}

// store_face_side for the packed lane: cell 0 is the low half of register
// 0, cell 7 the high half of register 3
template <int N, int SIDE, int A = 1>
__device__ __forceinline__ void store_face_side_h8(uint16_t* __restrict__ f, uint64_t row, uint32_t jk,
                                                   const uint32_t (*q)[4]) {
  if constexpr (ex(A) == SIDE)
    f[xface_index<__half, N, A>(row, jk)] = uint16_t(SIDE < 0 ? (q[A][0] & 0xFFFFu) : (q[A][3] >> 16));
  if constexpr (A + 1 < 19) store_face_side_h8<N, SIDE, A + 1>(f, row, jk, q);
}

template <int N, bool SIMPLE, bool TRT, bool INTERP>
__device__ __forceinline__ void update_lane_h8(const SweepArgs& a, const SlotCache& sc, int slot, uint32_t fl,
                                               int cell0) {
  constexpr int N3 = N * N * N;
  const int i0 = cell0 & (N - 1), j = (cell0 / N) & (N - 1), k = cell0 / (N * N);
  uint32_t q[19][4];
  uint32_t edge[kXDirs];
  uint32_t odd = 0;
  issue_all_h8<N, SIMPLE>(a, sc, slot, i0, j, k, q, edge, odd);
  shift_all_h8<N>(i0, q, edge);
  if (!SIMPLE && odd) fixups_h8<N, INTERP>(a, sc, slot, nbr_masks(sc), fl, i0, j, k, q);
  if (a.collide) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      float h[19][2];
#pragma unroll
      for (int d = 0; d < 19; ++d) h[d][0] = half_lo(q[d][p]), h[d][1] = half_hi(q[d][p]);
      collide_cell<__half, TRT>(a, h, 0);
      collide_cell<__half, TRT>(a, h, 1);
#pragma unroll
      for (int d = 0; d < 19; ++d) q[d][p] = pack_pair(h[d][0], h[d][1]);
    }
  }
  uint16_t* __restrict__ nxt = static_cast<uint16_t*>(a.nxt) + pdf_index<N>(0, uint32_t(slot), uint32_t(cell0));
#pragma unroll
  for (int d = 0; d < 19; ++d) {
    const u32x4 t = {q[d][0], q[d][1], q[d][2], q[d][3]};
    __builtin_nontemporal_store(t, reinterpret_cast<u32x4*>(nxt + d * N3));
  }
  if (a.face_out) {  // x-face copy (see store_faces)
    uint16_t* __restrict__ f = static_cast<uint16_t*>(a.face_out);
    const uint32_t jk = uint32_t(j + N * k);
    if (i0 == 0) store_face_side_h8<N, -1>(f, uint64_t(slot), jk, q);
    if (i0 == N - 8) store_face_side_h8<N, 1>(f, uint64_t(slot), jk, q);
  }
}

template <typename S, int N, bool SIMPLE, bool TRT, bool INTERP>
__device__ __forceinline__ void update_any(const SweepArgs& a, const SlotCache& sc, int slot, uint32_t fl, int cell0) {
  if constexpr (Geo<S, N>::PACKED)
    update_lane_h8<N, SIMPLE, TRT, INTERP>(a, sc, slot, fl, cell0);
  else
    update_lane<S, N, SIMPLE, TRT, INTERP>(a, sc, slot, fl, cell0);
}

// Work unit w: part w % SPLIT of work tile w / SPLIT (a tile split into
// SPLIT consecutive runs of whole rows, one per workgroup of T / SPLIT
// lanes).
template <typename S, int N, int SPLIT, bool TRT, bool INTERP>
__device__ __forceinline__ void sweep_item(const SweepArgs& a, int w) {
  constexpr int W = Geo<S, N>::W, CELLS = Geo<S, N>::CELLS, TPB = Geo<S, N>::TPB;
  const int item = a.work ? a.work[w / SPLIT] : a.work0 + w / SPLIT;
  const int slot = __builtin_amdgcn_readfirstlane(item / TPB);
  const int cell0 = (item - slot * TPB) * CELLS + (w % SPLIT) * (CELLS / SPLIT) + int(threadIdx.x) * W;
  // the slot's table, flags and fine row: loads of uniform addresses that
  // do not depend on each other, all in flight together
  SlotCache sc;
  const int32_t* nb = a.nbr + int64_t(slot) * 27;
#pragma unroll
  for (int q = 0; q < 27; ++q) sc.nbr[q] = __builtin_amdgcn_readfirstlane(nb[q]);
  const uint32_t fl = uint32_t(__builtin_amdgcn_readfirstlane(int(a.flags[slot])));
  const int row = __builtin_amdgcn_readfirstlane(a.fine_index[slot]);
  if ((fl & kHasFine) && row < 0 && threadIdx.x == 0) atomicOr(a.err, kErrNoChild);
  sc.fine_row = (fl & kHasFine) && row >= 0 ? row : 0;
  if (fl & kAllSameLevel)
    update_any<S, N, true, TRT, INTERP>(a, sc, slot, fl, cell0);
  else
    update_any<S, N, false, TRT, INTERP>(a, sc, slot, fl, cell0);
}

// Workgroup splits that keep at least one full wavefront per workgroup.
template <typename S, int N, int SPLIT>
constexpr bool split_ok() {
  return SPLIT == 1 || (Geo<S, N>::T / SPLIT >= 64 && (Geo<S, N>::CELLS / SPLIT) % N == 0);
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b to
// XCD b % 8), each XCD with its own L2.  xcd_unit maps workgroup b to a work
// unit such that every XCD sweeps one contiguous range of units: the halo
// rows that neighbouring tiles (and the parts of one tile) share then meet
// in the same L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_unit(int b, int n) {
  const int x = b & 7, r = b >> 3, q = n >> 3, rem = n & 7;
  return x * q + (x < rem ? x : rem) + r;
}

// One workgroup per work unit (PERSIST = false), or a fixed grid of
// workgroups looping over the units (PERSIST = true).  TRT: the TRT
// collision with a body force instead of SRT.  FUSED: the launch also runs
// the coarser level's coalescence (SweepArgs::fc), one chunk per workgroup
// at every fc_stride-th position of the first fc.nchunks * fc_stride; the
// other workgroups take the work units in order.  The chunks thus run
// while the sweep streams, instead of in a launch of their own; with
// fc_stride = 1 mod 8, chunk j runs on XCD j mod 8 as in a launch of its
// own (see kXcds).
template <typename S, int N, bool PERSIST, int SPLIT, bool TRT = false, bool INTERP = false, bool FUSED = false>
__global__ void __launch_bounds__((Geo<S, N>::T / SPLIT)) sweep_kernel(SweepArgs a) {
  const int units = a.nwork * SPLIT;
  if (!PERSIST) {
    int b = int(blockIdx.x);
    if constexpr (FUSED) {
      const int K = a.fc.nchunks, s = a.fc_stride;
      if (b % s == s - 1 && b / s < K) {
        __shared__ int32_t fns[8 * 27];
        __shared__ int32_t nbs[27];
        if (a.fc.walls)
          coalesce_chunk<S, N, false, true>(a.fc, b / s, fns, nbs);
        else
          coalesce_chunk<S, N, false, false>(a.fc, b / s, fns, nbs);
        return;
      }
      b -= min(K, (b + 1) / s);
    }
    sweep_item<S, N, SPLIT, TRT, INTERP>(a, a.xcd ? xcd_unit(b, units) : b);
    return;
  }
  for (int w = blockIdx.x; w < units; w += gridDim.x) sweep_item<S, N, SPLIT, TRT, INTERP>(a, a.xcd ? xcd_unit(w, units) : w);
}

// Largest split <= `requested` (1, 2 or 4) valid for storage S and n.
template <typename S>
int sweep_split_t(int n, int requested) {
  auto best = [&](auto nn) -> int {
    constexpr int N = decltype(nn)::value;
    if (requested >= 4 && split_ok<S, N, 4>()) return 4;
    if (requested >= 2 && split_ok<S, N, 2>()) return 2;
    return 1;
  };
  switch (n) {
    case 4: return best(std::integral_constant<int, 4>{});
    case 8: return best(std::integral_constant<int, 8>{});
    case 16: return best(std::integral_constant<int, 16>{});
    case 32: return best(std::integral_constant<int, 32>{});
    default: return 1;
  }
}

// Launch of one level substep for storage type S: `split` must be the value
// sweep_split_t returns, grid >= nwork * split launches one workgroup per
// work unit, a smaller grid a persistent one (SRT only: the TRT form always
// launches one workgroup per work unit).  With a.fc.nchunks > 0 (one
// workgroup per work unit and the homogeneous explosion only) the launch
// also runs those coalescence chunks, spread evenly over the grid.
template <typename S>
hipError_t launch_sweep_t(int n, const SweepArgs& a, int grid, int split, hipStream_t stream) {
  auto go = [&](auto nn, auto ss) -> hipError_t {
    constexpr int N = decltype(nn)::value, SPLIT = decltype(ss)::value;
    if constexpr (!split_ok<S, N, SPLIT>()) {
      return hipErrorInvalidValue;
    } else {
      constexpr int T = Geo<S, N>::T / SPLIT;
      if (a.fc.nchunks > 0) {
        const int units = a.nwork * SPLIT, K = a.fc.nchunks;
        if (a.interp || grid < units || units < 1) return hipErrorInvalidValue;
        // chunk positions j * s + s - 1 (j < K) stay inside the grid of
        // units + K workgroups for any s <= units / K + 1
        const int q = units / K;
        SweepArgs f = a;
        f.fc_stride = q >= 8 ? 8 * (q / 8) + 1 : 1;
        if (a.trt)
          hipLaunchKernelGGL((sweep_kernel<S, N, false, SPLIT, true, false, true>), dim3(units + K), dim3(T), 0, stream, f);
        else
          hipLaunchKernelGGL((sweep_kernel<S, N, false, SPLIT, false, false, true>), dim3(units + K), dim3(T), 0, stream, f);
        return hipGetLastError();
      }
      if (a.interp) {
        // the interpolated explosion: one workgroup of the full tile per work tile
        constexpr int T1 = Geo<S, N>::T;
        if (a.trt)
          hipLaunchKernelGGL((sweep_kernel<S, N, false, 1, true, true>), dim3(a.nwork), dim3(T1), 0, stream, a);
        else
          hipLaunchKernelGGL((sweep_kernel<S, N, false, 1, false, true>), dim3(a.nwork), dim3(T1), 0, stream, a);
      } else if (a.trt)
        hipLaunchKernelGGL((sweep_kernel<S, N, false, SPLIT, true>), dim3(a.nwork * SPLIT), dim3(T), 0, stream, a);
      else if (grid < a.nwork * SPLIT)
        hipLaunchKernelGGL((sweep_kernel<S, N, true, SPLIT>), dim3(grid), dim3(T), 0, stream, a);
      else
        hipLaunchKernelGGL((sweep_kernel<S, N, false, SPLIT>), dim3(a.nwork * SPLIT), dim3(T), 0, stream, a);
      return hipGetLastError();
    }
  };
  auto by_split = [&](auto nn) -> hipError_t {
    switch (split) {
      case 1: return go(nn, std::integral_constant<int, 1>{});
      case 2: return go(nn, std::integral_constant<int, 2>{});
      case 4: return go(nn, std::integral_constant<int, 4>{});
      default: return hipErrorInvalidValue;
    }
  };
  switch (n) {
    case 4: return by_split(std::integral_constant<int, 4>{});
    case 8: return by_split(std::integral_constant<int, 8>{});
    case 16: return by_split(std::integral_constant<int, 16>{});
    case 32: return by_split(std::integral_constant<int, 32>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dev
}  // namespace lbm
