// In-place streaming (AA pattern) kernels: the odd and even launches and the
// layout conversions (layouts and ownership in inplace.hpp).
//
// Work decomposition as in the two-buffer sweep: one workgroup per tile of
// one block, each lane W x-consecutive cells of one row (W = the storage
// form's 16-byte vector; packed FP16 pairs, 8 cells, for FP16 blocks of 8 or
// more cells per row), x shifts by one cell as DPP
// moves between the lanes of a row.  The even launch touches only the
// lane's own cells.  The odd launch reads and writes the lane's
// neighbours: rows shifted in y and z are whole vectors in the neighbour
// block (found in the scalar neighbour table), rows shifted in x come from
// the adjacent lane, and at a block's x face one element per row end
// crosses to the x neighbour: read from the x-face copy that the even
// launch wrote, and written to the entry buffer (same layout), which the
// even launch reads for the cells at x faces.  Every buffer row is then
// written with whole vectors.
#include "inplace.hpp"
#include "inplace_save.hpp"
#include "sweep.hpp"

namespace lbm {
namespace dev {

// Cells per lane as in the two-buffer sweep: FP16 blocks of 8 or more
// cells per row keep 8 cells per lane as packed half pairs (16-byte
// accesses, the packed launches below); otherwise the storage form's vector.
template <typename S, int N>
struct IGeo {
  static constexpr bool PACKED = sizeof(S) == 2 && N >= 8;
  static constexpr int W = PACKED ? 8 : Vec<S>::W;
  static constexpr int N3 = N * N * N;
  static constexpr int CELLS = N3 < 256 * W ? N3 : 256 * W;  // cells per workgroup
  static constexpr int T = CELLS / W;                          // lanes per workgroup
  static constexpr int TPB = N3 / CELLS;                       // tiles per block
  static_assert(N % W == 0 && N / W <= 16, "a cell row must fit one DPP row");
};

template <typename S>
struct IParm;
template <>
struct IParm<double> {
  static __device__ __forceinline__ double om(const InplaceArgs& a) { return a.omega64; }
  static __device__ __forceinline__ double lo(const InplaceArgs& a) { return a.lambda_o64; }
  static __device__ __forceinline__ double ac(const InplaceArgs& a, int d) { return a.accel64[d]; }
};
template <typename S>
struct IParm {
  static __device__ __forceinline__ float om(const InplaceArgs& a) { return a.omega; }
  static __device__ __forceinline__ float lo(const InplaceArgs& a) { return a.lambda_o; }
  static __device__ __forceinline__ float ac(const InplaceArgs& a, int d) { return a.accel[d]; }
};

template <typename S, bool TRT, typename C, int W>
__device__ __forceinline__ void icollide(const InplaceArgs& a, C (*h)[W], int c) {
  using P = IParm<S>;
  if constexpr (TRT)
    collide_trt<C, W>(h, c, C(P::om(a)), C(P::lo(a)), C(P::ac(a, 0)), C(P::ac(a, 1)), C(P::ac(a, 2)));
  else
    collide<C, W>(h, c, C(P::om(a)));
}

// The tile of workgroup b: block slot (wave-uniform) and the lane's first cell.
template <typename S, int N>
__device__ __forceinline__ void tile_of(const InplaceArgs& a, int& slot, int& cell0) {
  constexpr int TPB = IGeo<S, N>::TPB, CELLS = IGeo<S, N>::CELLS, W = IGeo<S, N>::W;
  const int units = a.nblocks * TPB;
  const int b = int(blockIdx.x);
  const int unit = a.xcd ? xcd_unit(b, units) : b;
  slot = __builtin_amdgcn_readfirstlane(unit / TPB);
  cell0 = (unit - slot * TPB) * CELLS + int(threadIdx.x) * W;
}

__device__ __forceinline__ void load_table(const InplaceArgs& a, int slot, SlotCache& sc) {
  const int32_t* nb = a.nbr + int64_t(slot) * 27;
#pragma unroll
  for (int q = 0; q < 27; ++q) sc.nbr[q] = __builtin_amdgcn_readfirstlane(nb[q]);
  sc.fine_row = 0;
}

// ---- odd launch: swapped -> pushed ------------------------------------------

// Issue the loads of direction A: f*_A(x - e_A) sits at (x - e_A, opp(A)).
// Bit A of `wall` marks a source beyond a wall for some cell of the lane.
template <typename S, int N, int A>
__device__ __forceinline__ void odd_issue(const InplaceArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                          typename Form<S>::C (*h)[IGeo<S, N>::W], typename Form<S>::C* edge,
                                          uint32_t& wall) {
  constexpr int W = IGeo<S, N>::W;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const int sy = j - EY, sz = k - EZ;
  const bool by = outside<N>(sy), bz = outside<N>(sz);
  const uint32_t row = uint32_t(N * ((sy & (N - 1)) + N * (sz & (N - 1))));
  const int nbm = pick<0, -EY, -EZ>(sc, false, by, bz);
  wall |= uint32_t(nbm < 0) << A;
  const S* __restrict__ buf = static_cast<const S*>(a.buf);
  Vec<S>::load(buf + pdf_index<N>(opp(A), uint32_t(nbm >= 0 ? nbm : slot), row + uint32_t(i0)), h[A]);
  if constexpr (EX != 0) {
    const bool at_end = EX == 1 ? i0 == 0 : i0 == N - W;
    const int nbx = pick<-EX, -EY, -EZ>(sc, true, by, bz);
    wall |= uint32_t(at_end && nbx < 0) << A;
    // f*_A of the x neighbour's end cell: the value leaving it through its x face
    const int eb = nbx >= 0 ? nbx : slot;
    edge[xdir_index(A)] = Form<S>::ld(static_cast<const S*>(a.face) + xface_index<S, N, A>(uint32_t(eb), row / N));
  }
}

template <typename S, int N, int A = 0>
__device__ __forceinline__ void odd_issue_all(const InplaceArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                              typename Form<S>::C (*h)[IGeo<S, N>::W], typename Form<S>::C* edge,
                                              uint32_t& wall) {
  odd_issue<S, N, A>(a, sc, slot, i0, j, k, h, edge, wall);
  if constexpr (A + 1 < 19) odd_issue_all<S, N, A + 1>(a, sc, slot, i0, j, k, h, edge, wall);
}

template <typename S, int N, int A = 0>
__device__ __forceinline__ void odd_shift_all(int i0, typename Form<S>::C (*h)[IGeo<S, N>::W],
                                              const typename Form<S>::C* edge) {
  using C = typename Form<S>::C;
  constexpr int W = IGeo<S, N>::W;
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
  if constexpr (A + 1 < 19) odd_shift_all<S, N, A + 1>(i0, h, edge);
}

// Sources beyond a wall: the cell's own post-collision value of the
// opposite direction, f*_opp(A)(x) (halfway bounce-back), which the swapped
// layout keeps at (x, A), and the x-face copy too where x is at an x face.
template <typename S, int N, int A = 1>
__device__ __forceinline__ void odd_walls(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0, int j,
                                          int k, uint32_t wall, typename Form<S>::C (*h)[IGeo<S, N>::W]) {
  constexpr int W = IGeo<S, N>::W;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  if ((wall >> A) & 1u) {
    const int sy = j - EY, sz = k - EZ;
    const bool by = outside<N>(sy), bz = outside<N>(sz);
    uint32_t cells = 0;
    if (pick<0, -EY, -EZ>(sc, false, by, bz) < 0) {
      cells = (1u << W) - 1u;
    } else if constexpr (EX != 0) {
      const bool at_end = EX == 1 ? i0 == 0 : i0 == N - W;
      if (at_end && pick<-EX, -EY, -EZ>(sc, true, by, bz) < 0) cells = EX == 1 ? 1u : 1u << (W - 1);
    }
    const S* __restrict__ own = static_cast<const S*>(a.buf) + pdf_index<N>(A, uint32_t(slot), uint32_t(cell0));
    if (cells == (1u << W) - 1u) {
#pragma unroll
      for (int c = 0; c < W; ++c) h[A][c] = Form<S>::ld(own + c);
    } else if constexpr (EX != 0) {
      // the end cell at an x wall: its own value leaving through that face,
      // from the x-face copy (in the buffer, an x-crossing push of another
      // row may overwrite that location during this launch)
      if (cells)
        h[A][EX == 1 ? 0 : W - 1] =
            Form<S>::ld(static_cast<const S*>(a.face) + xface_index<S, N, opp(A)>(uint32_t(slot), uint32_t(j + N * k)));
    }
  }
  if constexpr (A + 1 < 19) odd_walls<S, N, A + 1>(a, sc, slot, cell0, i0, j, k, wall, h);
}

// Store direction A: f*_A(x) to (x + e_A, A), or to (x, opp(A)) where x + e_A
// lies beyond a wall.  A value entering a block through an x face (cell
// x = 0 with e_A,x = +1, x = n - 1 with e_A,x = -1) goes to the entry buffer
// instead; the lane that would write it into the buffer's row writes its
// whole vector, the entering position included, which then holds no value.
template <typename S, int N, int A>
__device__ __forceinline__ void odd_store(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0, int j,
                                          int k, typename Form<S>::C (*h)[IGeo<S, N>::W]) {
  using C = typename Form<S>::C;
  constexpr int W = IGeo<S, N>::W;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  constexpr int END = EX == 1 ? W - 1 : 0;  // the cell that leaves through the x face
  S* __restrict__ buf = static_cast<S*>(a.buf);
  S* __restrict__ entry = static_cast<S*>(a.entry);
  const int dy = j + EY, dz = k + EZ;
  const bool by = outside<N>(dy), bz = outside<N>(dz);
  const uint32_t row = uint32_t(N * ((dy & (N - 1)) + N * (dz & (N - 1))));
  const int nbd = pick<0, EY, EZ>(sc, false, by, bz);
  const bool leaving_lane = EX == 1 ? i0 == N - W : i0 == 0;
  // x shift of the row by one cell (DPP, every lane takes part)
  C v[W];
  if constexpr (EX == 1) {
    const C prev = dpp_move<kDppRowShr1>(h[A][W - 1]);
    v[0] = prev;
#pragma unroll
    for (int c = 1; c < W; ++c) v[c] = h[A][c - 1];
  } else if constexpr (EX == -1) {
    const C next = dpp_move<kDppRowShl1>(h[A][0]);
#pragma unroll
    for (int c = 0; c < W - 1; ++c) v[c] = h[A][c + 1];
    v[W - 1] = next;
  }
  if (nbd < 0) {  // the whole destination row lies beyond a wall: every cell reflects
    Vec<S>::store(buf + pdf_index<N>(opp(A), uint32_t(slot), uint32_t(cell0)), h[A]);
    if constexpr (EX != 0)
      if (leaving_lane)  // the end cell's reflection enters through its own x face
        Form<S>::st(entry + xface_index<S, N, opp(A)>(uint32_t(slot), uint32_t(j + N * k)), h[A][END]);
    return;
  }
  S* __restrict__ dst = buf + pdf_index<N>(A, uint32_t(nbd), row + uint32_t(i0));
  if constexpr (EX == 0) {
    Vec<S>::store(dst, h[A]);
  } else {
    Vec<S>::store(dst, v);
    if (leaving_lane) {
      const int nbx = pick<EX, EY, EZ>(sc, true, by, bz);
      if (nbx >= 0)
        Form<S>::st(entry + xface_index<S, N, A>(uint32_t(nbx), row / N), h[A][END]);
      else  // an x wall: the reflection enters through the cell's own face
        Form<S>::st(entry + xface_index<S, N, opp(A)>(uint32_t(slot), uint32_t(j + N * k)), h[A][END]);
    }
  }
}

// ---- the finest level of a refined forest -------------------------------------
//
// The level's neighbour table also holds coarse codes (cells of the coarser
// region, whose values the explosion gives, eq. ctof) besides slots and
// walls.  The in-place launches of such a level read those values from the
// parent level's current state (kept in two buffers) and save what the
// back-trace and the coarser level's coalescence need (inplace_save.hpp).

// Post-collision value of the level-(L-1) parent of level-L cell (lx, ly, lz)
// of the virtual block with coarse code `code` (homogeneous explosion).  A
// parent on the parent block's x face through which A leaves it is read
// from the parent's x-face copy (as parent_ptr in the sweep does).
template <typename S, int N, int A>
__device__ __forceinline__ const S* iparent(const InplaceArgs& a, int code, int lx, int ly, int lz) {
  constexpr int H = N / 2;
  const int pp = kNbrCoarse0 - code;
  const int oc = pp & 7;
  const int px = (oc & 1 ? H : 0) + (lx >> 1), py = (oc & 2 ? H : 0) + (ly >> 1), pz = (oc & 4 ? H : 0) + (lz >> 1);
  if constexpr (ex(A) != 0) {
    if (px == (ex(A) > 0 ? N - 1 : 0))
      return static_cast<const S*>(a.par_face) + xface_index<S, N, A>(uint32_t(pp >> 3), uint32_t(py + N * pz));
  }
  return static_cast<const S*>(a.par) + pdf_index<N>(A, uint32_t(pp >> 3), uint32_t(px + N * (py + N * pz)));
}

// Odd launch (the level's first substep): the source of every cell of the
// lane whose direction-A source is no cell of the level, from the exact
// table entry of that source: a wall gives the bounce-back (own (x, A), or
// the x-face copy at an x face, see odd_walls), a coarse code the exploded
// parent value.
template <typename S, int N, int A = 1>
__device__ __forceinline__ void odd_specials_ref(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0,
                                                 int j, int k, uint32_t special,
                                                 typename Form<S>::C (*h)[IGeo<S, N>::W]) {
  constexpr int W = IGeo<S, N>::W;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  if ((special >> A) & 1u) {
    const int sy = j - EY, sz = k - EZ;
    const bool by = outside<N>(sy), bz = outside<N>(sz);
    const S* p[W];
#pragma unroll
    for (int c = 0; c < W; ++c) {
      const int sx = i0 + c - EX;
      const int code = pick<-EX, -EY, -EZ>(sc, outside<N>(sx), by, bz);
      const int x = i0 + c;
      p[c] = nullptr;
      if (code == kNbrWall) {
        const bool xface = EX != 0 && x == (EX == 1 ? 0 : N - 1);
        p[c] = xface ? static_cast<const S*>(a.face) + xface_index<S, N, opp(A)>(uint32_t(slot), uint32_t(j + N * k))
                     : static_cast<const S*>(a.buf) + pdf_index<N>(A, uint32_t(slot), uint32_t(cell0 + c));
      } else if (code <= kNbrCoarse0) {
        p[c] = iparent<S, N, A>(a, code, sx & (N - 1), sy & (N - 1), sz & (N - 1));
      } else if (code < 0) {
        atomicOr(a.err, kErrNoSource);
      }
    }
#pragma unroll
    for (int c = 0; c < W; ++c)
      if (p[c]) h[A][c] = Form<S>::ld(p[c]);
  }
  if constexpr (A + 1 < 19) odd_specials_ref<S, N, A + 1>(a, sc, slot, cell0, i0, j, k, special, h);
}

// Odd-launch stores of the finest level: as odd_store, with the end cell of
// an x-shifted row sent by its own destination (the x-diagonal block, which
// may differ from the row's block), and every value whose destination lies
// in the coarser region also saved (t + 1/2).
template <typename S, int N, int A>
__device__ __forceinline__ void odd_store_ref(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0,
                                              int j, int k, typename Form<S>::C (*h)[IGeo<S, N>::W]) {
  using C = typename Form<S>::C;
  constexpr int W = IGeo<S, N>::W;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  constexpr int END = EX == 1 ? W - 1 : 0;
  S* __restrict__ buf = static_cast<S*>(a.buf);
  S* __restrict__ entry = static_cast<S*>(a.entry);
  S* __restrict__ save = static_cast<S*>(a.save_out);
  const int dy = j + EY, dz = k + EZ;
  const bool by = outside<N>(dy), bz = outside<N>(dz);
  const uint32_t row = uint32_t(N * ((dy & (N - 1)) + N * (dz & (N - 1))));
  const int nbd = pick<0, EY, EZ>(sc, false, by, bz);
  const bool leaving_lane = EX != 0 && (EX == 1 ? i0 == N - W : i0 == 0);
  C v[W];
  if constexpr (EX == 1) {
    const C prev = dpp_move<kDppRowShr1>(h[A][W - 1]);
    v[0] = prev;
#pragma unroll
    for (int c = 1; c < W; ++c) v[c] = h[A][c - 1];
  } else if constexpr (EX == -1) {
    const C next = dpp_move<kDppRowShl1>(h[A][0]);
#pragma unroll
    for (int c = 0; c < W - 1; ++c) v[c] = h[A][c + 1];
    v[W - 1] = next;
  } else {
#pragma unroll
    for (int c = 0; c < W; ++c) v[c] = h[A][c];
  }
  if (nbd < 0) {
    // the row's destination is no cell of the level: every cell reflects
    // (a coarse destination's reflection slot is never read)
    Vec<S>::store(buf + pdf_index<N>(opp(A), uint32_t(slot), uint32_t(cell0)), h[A]);
    if (nbd <= kNbrCoarse0) {
#pragma unroll
      for (int c = 0; c < W; ++c)
        if (!(leaving_lane && c == END))
          Form<S>::st(save + save_index<N>(uint32_t(slot), A, i0 + c, j, k), h[A][c]);
    }
  } else {
    Vec<S>::store(buf + pdf_index<N>(A, uint32_t(nbd), row + uint32_t(i0)), v);
  }
  if constexpr (EX != 0) {
    if (leaving_lane) {
      const int nbx = pick<EX, EY, EZ>(sc, true, by, bz);
      if (nbx >= 0) {
        Form<S>::st(entry + xface_index<S, N, A>(uint32_t(nbx), row / N), h[A][END]);
      } else {
        Form<S>::st(entry + xface_index<S, N, opp(A)>(uint32_t(slot), uint32_t(j + N * k)), h[A][END]);
        if (nbx <= kNbrCoarse0) Form<S>::st(save + save_index<N>(uint32_t(slot), A, i0 + END, j, k), h[A][END]);
      }
    }
  }
}

template <typename S, int N, bool REF, int A = 0>
__device__ __forceinline__ void odd_store_all(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0,
                                              int j, int k, typename Form<S>::C (*h)[IGeo<S, N>::W]) {
  if constexpr (REF)
    odd_store_ref<S, N, A>(a, sc, slot, cell0, i0, j, k, h);
  else
    odd_store<S, N, A>(a, sc, slot, cell0, i0, j, k, h);
  if constexpr (A + 1 < 19) odd_store_all<S, N, REF, A + 1>(a, sc, slot, cell0, i0, j, k, h);
}

// REF: the finest level of a refined forest (coarse neighbours; explosion
// and saves), else a forest of one level.
template <typename S, int N, bool TRT, bool REF>
__global__ void __launch_bounds__((IGeo<S, N>::T)) inplace_odd_kernel(InplaceArgs a) {
  using C = typename Form<S>::C;
  constexpr int W = IGeo<S, N>::W;
  int slot, cell0;
  tile_of<S, N>(a, slot, cell0);
  SlotCache sc;
  load_table(a, slot, sc);
  const int i0 = cell0 & (N - 1), j = (cell0 / N) & (N - 1), k = cell0 / (N * N);
  C h[19][W];
  C edge[kXDirs];
  uint32_t wall = 0;
  odd_issue_all<S, N>(a, sc, slot, i0, j, k, h, edge, wall);
  odd_shift_all<S, N>(i0, h, edge);
  if constexpr (REF) {
    if (wall) odd_specials_ref<S, N>(a, sc, slot, cell0, i0, j, k, wall, h);
  } else {
    if (wall) odd_walls<S, N>(a, sc, slot, cell0, i0, j, k, wall, h);
  }
#pragma unroll
  for (int c = 0; c < W; ++c) icollide<S, TRT>(a, h, c);
  odd_store_all<S, N, REF>(a, sc, slot, cell0, i0, j, k, h);
}

// ---- even launch: pushed -> swapped -------------------------------------------

// Even launch (the level's second substep) on the finest level: a cell
// whose direction-A source x - e_A lies in the coarser region takes what the
// first substep streamed into that ghost cell: the level's own state at t at
// x - 2 e_A (saved), or the exploded parent value (of the opposite direction
// if x - 2 e_A is a wall: the ghost cell's bounce-back).
template <typename S, int N, int A = 1>
__device__ __forceinline__ void even_specials_ref(const InplaceArgs& a, const SlotCache& sc, int i0, int j, int k,
                                                  typename Form<S>::C (*h)[IGeo<S, N>::W]) {
  constexpr int W = IGeo<S, N>::W;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const int sy = j - EY, sz = k - EZ, zy = sy - EY, zz = sz - EZ;
  const bool by = outside<N>(sy), bz = outside<N>(sz), bzy = outside<N>(zy), bzz = outside<N>(zz);
  const S* p[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int sx = i0 + c - EX, zx = sx - EX;
    const int code = pick<-EX, -EY, -EZ>(sc, outside<N>(sx), by, bz);
    p[c] = nullptr;
    if (code <= kNbrCoarse0) {
      const int cz = pick<-EX, -EY, -EZ>(sc, outside<N>(zx), bzy, bzz);
      if (cz >= 0)
        p[c] = static_cast<const S*>(a.save_in) +
               save_index<N>(uint32_t(cz), A, zx & (N - 1), zy & (N - 1), zz & (N - 1));
      else if (cz == kNbrWall)
        p[c] = iparent<S, N, opp(A)>(a, code, sx & (N - 1), sy & (N - 1), sz & (N - 1));
      else if (cz <= kNbrCoarse0)
        p[c] = iparent<S, N, A>(a, cz, zx & (N - 1), zy & (N - 1), zz & (N - 1));
      else
        atomicOr(a.err, kErrNoSource);
    }
  }
#pragma unroll
  for (int c = 0; c < W; ++c)
    if (p[c]) h[A][c] = Form<S>::ld(p[c]);
  if constexpr (A + 1 < 19) even_specials_ref<S, N, A + 1>(a, sc, i0, j, k, h);
}

// Values of the finest level whose destination lies in the coarser region,
// saved at t + 1 for the next parent step's back-trace and coalescence.
template <typename S, int N, int A = 1>
__device__ __forceinline__ void even_saves_ref(const InplaceArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                               const typename Form<S>::C (*h)[IGeo<S, N>::W]) {
  constexpr int W = IGeo<S, N>::W;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  S* __restrict__ save = static_cast<S*>(a.save_out);
  const int dy = j + EY, dz = k + EZ;
  const bool by = outside<N>(dy), bz = outside<N>(dz);
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int code = pick<EX, EY, EZ>(sc, outside<N>(i0 + c + EX), by, bz);
    if (code <= kNbrCoarse0) Form<S>::st(save + save_index<N>(uint32_t(slot), A, i0 + c, j, k), h[A][c]);
  }
  if constexpr (A + 1 < 19) even_saves_ref<S, N, A + 1>(a, sc, slot, i0, j, k, h);
}

template <typename S, int N, bool TRT, bool REF>
__global__ void __launch_bounds__((IGeo<S, N>::T)) inplace_even_kernel(InplaceArgs a) {
  using C = typename Form<S>::C;
  constexpr int W = IGeo<S, N>::W, N3 = N * N * N;
  int slot, cell0;
  tile_of<S, N>(a, slot, cell0);
  const int i0 = cell0 & (N - 1), j = (cell0 / N) & (N - 1), k = cell0 / (N * N);
  S* __restrict__ p = static_cast<S*>(a.buf) + pdf_index<N>(0, uint32_t(slot), uint32_t(cell0));
  C h[19][W];
#pragma unroll
  for (int d = 0; d < 19; ++d) Vec<S>::load(p + d * N3, h[d]);
  // values that entered through an x face come from the entry buffer
  const S* __restrict__ e = static_cast<const S*>(a.entry);
  const uint32_t jk0 = uint32_t(j + N * k);
#pragma unroll
  for (int d = 1; d < 19; ++d) {
    if (ex(d) == 1 && i0 == 0) h[d][0] = Form<S>::ld(e + xface_at<S, N>(uint64_t(slot), xdir_index_rt(d), jk0));
    if (ex(d) == -1 && i0 == N - W) h[d][W - 1] = Form<S>::ld(e + xface_at<S, N>(uint64_t(slot), xdir_index_rt(d), jk0));
  }
  bool coarse_nbr = false;
  SlotCache sc;
  if constexpr (REF) {
    coarse_nbr = (__builtin_amdgcn_readfirstlane(int(a.flags[slot])) & int(kHasCoarse)) != 0;
    if (coarse_nbr) {
      load_table(a, slot, sc);
      even_specials_ref<S, N>(a, sc, i0, j, k, h);
    }
  }
#pragma unroll
  for (int c = 0; c < W; ++c) icollide<S, TRT>(a, h, c);
#pragma unroll
  for (int d = 0; d < 19; ++d) Vec<S>::store(p + opp(d) * N3, h[d]);
  if constexpr (REF) {
    if (coarse_nbr) even_saves_ref<S, N>(a, sc, slot, i0, j, k, h);
  }
  // x-face copy for the next odd launch: the values leaving the block
  // through its x faces, by direction
  S* __restrict__ f = static_cast<S*>(a.face);
  const uint32_t jk = uint32_t(j + N * k);
#pragma unroll
  for (int d = 1; d < 19; ++d) {
    if (ex(d) == 1 && i0 == N - W) Form<S>::st(f + xface_at<S, N>(uint64_t(slot), xdir_index_rt(d), jk), h[d][W - 1]);
    if (ex(d) == -1 && i0 == 0) Form<S>::st(f + xface_at<S, N>(uint64_t(slot), xdir_index_rt(d), jk), h[d][0]);
  }
}

// ---- packed FP16 launches (8 cells per lane as 4 registers of half pairs) --
//
// Register r of direction A holds cells 2r (low half) and 2r + 1 (high
// half) of the lane's row segment, as in the two-buffer sweep's packed path;
// a shift by one cell is a 16-bit funnel shift of neighbouring registers,
// the register across the lane boundary coming from a DPP move.  Each pair
// is unpacked to FP32 for its collision, exactly as the two-buffer sweep
// does, so both round identically.

template <bool TRT>
__device__ __forceinline__ void collide_h8(const InplaceArgs& a, uint32_t (*q)[4]) {
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    float h[19][2];
#pragma unroll
    for (int d = 0; d < 19; ++d) h[d][0] = half_lo(q[d][p]), h[d][1] = half_hi(q[d][p]);
    icollide<__half, TRT>(a, h, 0);
    icollide<__half, TRT>(a, h, 1);
#pragma unroll
    for (int d = 0; d < 19; ++d) q[d][p] = pack_pair(h[d][0], h[d][1]);
  }
}

// the 8 cells shifted by one position: EX = +1 gives position c the cell
// c - 1 (position 0 from `in`, the previous lane's last register), EX = -1
// the cell c + 1 (position 7 from `in`, the next lane's first register)
template <int EX>
__device__ __forceinline__ void shift_h8(const uint32_t* q, uint32_t in, uint32_t* o) {
  if constexpr (EX == 1) {
    o[3] = funnel16(q[3], q[2]);
    o[2] = funnel16(q[2], q[1]);
    o[1] = funnel16(q[1], q[0]);
    o[0] = funnel16(q[0], in);
  } else {
    o[0] = funnel16(q[1], q[0]);
    o[1] = funnel16(q[2], q[1]);
    o[2] = funnel16(q[3], q[2]);
    o[3] = funnel16(in, q[3]);
  }
}

template <int N, int A>
__device__ __forceinline__ void odd_issue_h8(const InplaceArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                             uint32_t (*q)[4], uint32_t* edge, uint32_t& wall) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const int sy = j - EY, sz = k - EZ;
  const bool by = outside<N>(sy), bz = outside<N>(sz);
  const uint32_t row = uint32_t(N * ((sy & (N - 1)) + N * (sz & (N - 1))));
  const int nbm = pick<0, -EY, -EZ>(sc, false, by, bz);
  wall |= uint32_t(nbm < 0) << A;
  const uint16_t* __restrict__ buf = static_cast<const uint16_t*>(a.buf);
  const uint4 v =
      *reinterpret_cast<const uint4*>(buf + pdf_index<N>(opp(A), uint32_t(nbm >= 0 ? nbm : slot), row + uint32_t(i0)));
  q[A][0] = v.x, q[A][1] = v.y, q[A][2] = v.z, q[A][3] = v.w;
  if constexpr (EX != 0) {
    const bool at_end = EX == 1 ? i0 == 0 : i0 == N - 8;
    const int nbx = pick<-EX, -EY, -EZ>(sc, true, by, bz);
    wall |= uint32_t(at_end && nbx < 0) << A;
    const int eb = nbx >= 0 ? nbx : slot;
    edge[xdir_index(A)] = static_cast<const uint16_t*>(a.face)[xface_index<__half, N, A>(uint32_t(eb), row / N)];
  }
}

template <int N, int A = 0>
__device__ __forceinline__ void odd_issue_all_h8(const InplaceArgs& a, const SlotCache& sc, int slot, int i0, int j,
                                                 int k, uint32_t (*q)[4], uint32_t* edge, uint32_t& wall) {
  odd_issue_h8<N, A>(a, sc, slot, i0, j, k, q, edge, wall);
  if constexpr (A + 1 < 19) odd_issue_all_h8<N, A + 1>(a, sc, slot, i0, j, k, q, edge, wall);
}

template <int N, int A = 0>
__device__ __forceinline__ void odd_shift_all_h8(int i0, uint32_t (*q)[4], const uint32_t* edge) {
  constexpr int EX = ex(A);
  if constexpr (EX == 1) {  // cell c takes cell c - 1
    const uint32_t prev = dpp_move_u32<kDppRowShr1>(q[A][3]);
    uint32_t o[4];
    shift_h8<1>(q[A], i0 == 0 ? edge[xdir_index(A)] << 16 : prev, o);
#pragma unroll
    for (int r = 0; r < 4; ++r) q[A][r] = o[r];
  } else if constexpr (EX == -1) {  // cell c takes cell c + 1
    const uint32_t next = dpp_move_u32<kDppRowShl1>(q[A][0]);
    uint32_t o[4];
    shift_h8<-1>(q[A], i0 == N - 8 ? edge[xdir_index(A)] : next, o);
#pragma unroll
    for (int r = 0; r < 4; ++r) q[A][r] = o[r];
  }
  if constexpr (A + 1 < 19) odd_shift_all_h8<N, A + 1>(i0, q, edge);
}

// sources beyond a wall: the cell's own (x, A) in the swapped layout
template <int N, int A = 1>
__device__ __forceinline__ void odd_walls_h8(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0,
                                             int j, int k, uint32_t wall, uint32_t (*q)[4]) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  if ((wall >> A) & 1u) {
    const int sy = j - EY, sz = k - EZ;
    const bool by = outside<N>(sy), bz = outside<N>(sz);
    const uint16_t* __restrict__ own =
        static_cast<const uint16_t*>(a.buf) + pdf_index<N>(A, uint32_t(slot), uint32_t(cell0));
    if (pick<0, -EY, -EZ>(sc, false, by, bz) < 0) {
      const uint4 v = *reinterpret_cast<const uint4*>(own);
      q[A][0] = v.x, q[A][1] = v.y, q[A][2] = v.z, q[A][3] = v.w;
    } else if constexpr (EX != 0) {
      const bool at_end = EX == 1 ? i0 == 0 : i0 == N - 8;
      if (at_end && pick<-EX, -EY, -EZ>(sc, true, by, bz) < 0) {  // from the x-face copy (see odd_walls)
        const uint32_t v =
            static_cast<const uint16_t*>(a.face)[xface_index<__half, N, opp(A)>(uint32_t(slot), uint32_t(j + N * k))];
        if (EX == 1)
          q[A][0] = (q[A][0] & 0xFFFF0000u) | v;
        else
          q[A][3] = (q[A][3] & 0xFFFFu) | (v << 16);
      }
    }
  }
  if constexpr (A + 1 < 19) odd_walls_h8<N, A + 1>(a, sc, slot, cell0, i0, j, k, wall, q);
}

__device__ __forceinline__ void store_u32x4(uint16_t* p, const uint32_t* o) {
  const u32x4 t = {o[0], o[1], o[2], o[3]};
  __builtin_nontemporal_store(t, reinterpret_cast<u32x4*>(p));
}

template <int N, int A>
__device__ __forceinline__ void odd_store_h8(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0, int j,
                                             int k, uint32_t (*q)[4]) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  uint16_t* __restrict__ buf = static_cast<uint16_t*>(a.buf);
  uint16_t* __restrict__ entry = static_cast<uint16_t*>(a.entry);
  const int dy = j + EY, dz = k + EZ;
  const bool by = outside<N>(dy), bz = outside<N>(dz);
  const uint32_t row = uint32_t(N * ((dy & (N - 1)) + N * (dz & (N - 1))));
  const int nbd = pick<0, EY, EZ>(sc, false, by, bz);
  const bool leaving_lane = EX == 1 ? i0 == N - 8 : i0 == 0;
  const uint16_t end = EX == 1 ? uint16_t(q[A][3] >> 16) : uint16_t(q[A][0] & 0xFFFFu);
  uint32_t o[4];
  if constexpr (EX == 1) {
    shift_h8<1>(q[A], dpp_move_u32<kDppRowShr1>(q[A][3]), o);
  } else if constexpr (EX == -1) {
    shift_h8<-1>(q[A], dpp_move_u32<kDppRowShl1>(q[A][0]), o);
  }
  if (nbd < 0) {  // the whole destination row lies beyond a wall: every cell reflects
    store_u32x4(buf + pdf_index<N>(opp(A), uint32_t(slot), uint32_t(cell0)), q[A]);
    if constexpr (EX != 0)
      if (leaving_lane) entry[xface_index<__half, N, opp(A)>(uint32_t(slot), uint32_t(j + N * k))] = end;
    return;
  }
  uint16_t* __restrict__ dst = buf + pdf_index<N>(A, uint32_t(nbd), row + uint32_t(i0));
  if constexpr (EX == 0) {
    store_u32x4(dst, q[A]);
  } else {
    store_u32x4(dst, o);
    if (leaving_lane) {
      const int nbx = pick<EX, EY, EZ>(sc, true, by, bz);
      if (nbx >= 0)
        entry[xface_index<__half, N, A>(uint32_t(nbx), row / N)] = end;
      else
        entry[xface_index<__half, N, opp(A)>(uint32_t(slot), uint32_t(j + N * k))] = end;
    }
  }
}

template <int N, int A = 0>
__device__ __forceinline__ void odd_store_all_h8(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0,
                                                 int j, int k, uint32_t (*q)[4]) {
  odd_store_h8<N, A>(a, sc, slot, cell0, i0, j, k, q);
  if constexpr (A + 1 < 19) odd_store_all_h8<N, A + 1>(a, sc, slot, cell0, i0, j, k, q);
}

// ---- packed FP16 on the finest level of a refined forest (as the REF paths above)

__device__ __forceinline__ void put_half(uint32_t* q, int c, uint16_t v) {
  uint32_t& w = q[c >> 1];
  w = c & 1 ? ((w & 0xFFFFu) | (uint32_t(v) << 16)) : ((w & 0xFFFF0000u) | uint32_t(v));
}
__device__ __forceinline__ uint16_t get_half(const uint32_t* q, int c) {
  return uint16_t(c & 1 ? q[c >> 1] >> 16 : q[c >> 1] & 0xFFFFu);
}

template <int N, int A = 1>
__device__ __forceinline__ void odd_specials_ref_h8(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0,
                                                    int j, int k, uint32_t special, uint32_t (*q)[4]) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  if ((special >> A) & 1u) {
    const int sy = j - EY, sz = k - EZ;
    const bool by = outside<N>(sy), bz = outside<N>(sz);
    const uint16_t* p[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int sx = i0 + c - EX;
      const int code = pick<-EX, -EY, -EZ>(sc, outside<N>(sx), by, bz);
      const int x = i0 + c;
      p[c] = nullptr;
      if (code == kNbrWall) {
        const bool xface = EX != 0 && x == (EX == 1 ? 0 : N - 1);
        p[c] = xface ? static_cast<const uint16_t*>(a.face) + xface_index<__half, N, opp(A)>(uint32_t(slot), uint32_t(j + N * k))
                     : static_cast<const uint16_t*>(a.buf) + pdf_index<N>(A, uint32_t(slot), uint32_t(cell0 + c));
      } else if (code <= kNbrCoarse0) {
        p[c] = reinterpret_cast<const uint16_t*>(iparent<__half, N, A>(a, code, sx & (N - 1), sy & (N - 1), sz & (N - 1)));
      } else if (code < 0) {
        atomicOr(a.err, kErrNoSource);
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (p[c]) put_half(q[A], c, *p[c]);
  }
  if constexpr (A + 1 < 19) odd_specials_ref_h8<N, A + 1>(a, sc, slot, cell0, i0, j, k, special, q);
}

template <int N, int A>
__device__ __forceinline__ void odd_store_ref_h8(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0,
                                                 int j, int k, uint32_t (*q)[4]) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  constexpr int END = EX == 1 ? 7 : 0;
  uint16_t* __restrict__ buf = static_cast<uint16_t*>(a.buf);
  uint16_t* __restrict__ entry = static_cast<uint16_t*>(a.entry);
  uint16_t* __restrict__ save = static_cast<uint16_t*>(a.save_out);
  const int dy = j + EY, dz = k + EZ;
  const bool by = outside<N>(dy), bz = outside<N>(dz);
  const uint32_t row = uint32_t(N * ((dy & (N - 1)) + N * (dz & (N - 1))));
  const int nbd = pick<0, EY, EZ>(sc, false, by, bz);
  const bool leaving_lane = EX != 0 && (EX == 1 ? i0 == N - 8 : i0 == 0);
  uint32_t o[4] = {q[A][0], q[A][1], q[A][2], q[A][3]};
  if constexpr (EX == 1) {
    shift_h8<1>(q[A], dpp_move_u32<kDppRowShr1>(q[A][3]), o);
  } else if constexpr (EX == -1) {
    shift_h8<-1>(q[A], dpp_move_u32<kDppRowShl1>(q[A][0]), o);
  }
  if (nbd < 0) {
    store_u32x4(buf + pdf_index<N>(opp(A), uint32_t(slot), uint32_t(cell0)), q[A]);
    if (nbd <= kNbrCoarse0) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (!(leaving_lane && c == END)) save[save_index<N>(uint32_t(slot), A, i0 + c, j, k)] = get_half(q[A], c);
    }
  } else {
    store_u32x4(buf + pdf_index<N>(A, uint32_t(nbd), row + uint32_t(i0)), o);
  }
  if constexpr (EX != 0) {
    if (leaving_lane) {
      const uint16_t end = get_half(q[A], END);
      const int nbx = pick<EX, EY, EZ>(sc, true, by, bz);
      if (nbx >= 0) {
        entry[xface_index<__half, N, A>(uint32_t(nbx), row / N)] = end;
      } else {
        entry[xface_index<__half, N, opp(A)>(uint32_t(slot), uint32_t(j + N * k))] = end;
        if (nbx <= kNbrCoarse0) save[save_index<N>(uint32_t(slot), A, i0 + END, j, k)] = end;
      }
    }
  }
}

template <int N, bool REF, int A = 0>
__device__ __forceinline__ void odd_store_sel_h8(const InplaceArgs& a, const SlotCache& sc, int slot, int cell0, int i0,
                                                 int j, int k, uint32_t (*q)[4]) {
  if constexpr (REF)
    odd_store_ref_h8<N, A>(a, sc, slot, cell0, i0, j, k, q);
  else
    odd_store_h8<N, A>(a, sc, slot, cell0, i0, j, k, q);
  if constexpr (A + 1 < 19) odd_store_sel_h8<N, REF, A + 1>(a, sc, slot, cell0, i0, j, k, q);
}

template <int N, int A = 1>
__device__ __forceinline__ void even_specials_ref_h8(const InplaceArgs& a, const SlotCache& sc, int i0, int j, int k,
                                                     uint32_t (*q)[4]) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const int sy = j - EY, sz = k - EZ, zy = sy - EY, zz = sz - EZ;
  const bool by = outside<N>(sy), bz = outside<N>(sz), bzy = outside<N>(zy), bzz = outside<N>(zz);
  const uint16_t* p[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int sx = i0 + c - EX, zx = sx - EX;
    const int code = pick<-EX, -EY, -EZ>(sc, outside<N>(sx), by, bz);
    p[c] = nullptr;
    if (code <= kNbrCoarse0) {
      const int cz = pick<-EX, -EY, -EZ>(sc, outside<N>(zx), bzy, bzz);
      if (cz >= 0)
        p[c] = static_cast<const uint16_t*>(a.save_in) +
               save_index<N>(uint32_t(cz), A, zx & (N - 1), zy & (N - 1), zz & (N - 1));
      else if (cz == kNbrWall)
        p[c] = reinterpret_cast<const uint16_t*>(iparent<__half, N, opp(A)>(a, code, sx & (N - 1), sy & (N - 1), sz & (N - 1)));
      else if (cz <= kNbrCoarse0)
        p[c] = reinterpret_cast<const uint16_t*>(iparent<__half, N, A>(a, cz, zx & (N - 1), zy & (N - 1), zz & (N - 1)));
      else
        atomicOr(a.err, kErrNoSource);
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (p[c]) put_half(q[A], c, *p[c]);
  if constexpr (A + 1 < 19) even_specials_ref_h8<N, A + 1>(a, sc, i0, j, k, q);
}

template <int N, int A = 1>
__device__ __forceinline__ void even_saves_ref_h8(const InplaceArgs& a, const SlotCache& sc, int slot, int i0, int j,
                                                  int k, const uint32_t (*q)[4]) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  uint16_t* __restrict__ save = static_cast<uint16_t*>(a.save_out);
  const int dy = j + EY, dz = k + EZ;
  const bool by = outside<N>(dy), bz = outside<N>(dz);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int code = pick<EX, EY, EZ>(sc, outside<N>(i0 + c + EX), by, bz);
    if (code <= kNbrCoarse0) save[save_index<N>(uint32_t(slot), A, i0 + c, j, k)] = get_half(q[A], c);
  }
  if constexpr (A + 1 < 19) even_saves_ref_h8<N, A + 1>(a, sc, slot, i0, j, k, q);
}

template <int N, bool TRT, bool REF>
__global__ void __launch_bounds__((IGeo<__half, N>::T)) inplace_odd_h8_kernel(InplaceArgs a) {
  int slot, cell0;
  tile_of<__half, N>(a, slot, cell0);
  SlotCache sc;
  load_table(a, slot, sc);
  const int i0 = cell0 & (N - 1), j = (cell0 / N) & (N - 1), k = cell0 / (N * N);
  uint32_t q[19][4];
  uint32_t edge[kXDirs];
  uint32_t wall = 0;
  odd_issue_all_h8<N>(a, sc, slot, i0, j, k, q, edge, wall);
  odd_shift_all_h8<N>(i0, q, edge);
  if constexpr (REF) {
    if (wall) odd_specials_ref_h8<N>(a, sc, slot, cell0, i0, j, k, wall, q);
  } else {
    if (wall) odd_walls_h8<N>(a, sc, slot, cell0, i0, j, k, wall, q);
  }
  collide_h8<TRT>(a, q);
  odd_store_sel_h8<N, REF>(a, sc, slot, cell0, i0, j, k, q);
}

template <int N, bool TRT, bool REF>
__global__ void __launch_bounds__((IGeo<__half, N>::T)) inplace_even_h8_kernel(InplaceArgs a) {
  constexpr int N3 = N * N * N;
  int slot, cell0;
  tile_of<__half, N>(a, slot, cell0);
  const int i0 = cell0 & (N - 1), j = (cell0 / N) & (N - 1), k = cell0 / (N * N);
  uint16_t* __restrict__ p = static_cast<uint16_t*>(a.buf) + pdf_index<N>(0, uint32_t(slot), uint32_t(cell0));
  uint32_t q[19][4];
#pragma unroll
  for (int d = 0; d < 19; ++d) {
    const uint4 v = *reinterpret_cast<const uint4*>(p + d * N3);
    q[d][0] = v.x, q[d][1] = v.y, q[d][2] = v.z, q[d][3] = v.w;
  }
  const uint16_t* __restrict__ e = static_cast<const uint16_t*>(a.entry);
  const uint32_t jk0 = uint32_t(j + N * k);
#pragma unroll
  for (int d = 1; d < 19; ++d) {  // values that entered through an x face
    if (ex(d) == 1 && i0 == 0)
      q[d][0] = (q[d][0] & 0xFFFF0000u) | uint32_t(e[xface_at<__half, N>(uint64_t(slot), xdir_index_rt(d), jk0)]);
    if (ex(d) == -1 && i0 == N - 8)
      q[d][3] = (q[d][3] & 0xFFFFu) | (uint32_t(e[xface_at<__half, N>(uint64_t(slot), xdir_index_rt(d), jk0)]) << 16);
  }
  bool coarse_nbr = false;
  SlotCache sc;
  if constexpr (REF) {
    coarse_nbr = (__builtin_amdgcn_readfirstlane(int(a.flags[slot])) & int(kHasCoarse)) != 0;
    if (coarse_nbr) {
      load_table(a, slot, sc);
      even_specials_ref_h8<N>(a, sc, i0, j, k, q);
    }
  }
  collide_h8<TRT>(a, q);
#pragma unroll
  for (int d = 0; d < 19; ++d) store_u32x4(p + opp(d) * N3, q[d]);
  if constexpr (REF) {
    if (coarse_nbr) even_saves_ref_h8<N>(a, sc, slot, i0, j, k, q);
  }
  uint16_t* __restrict__ f = static_cast<uint16_t*>(a.face);
  const uint32_t jk = uint32_t(j + N * k);
#pragma unroll
  for (int d = 1; d < 19; ++d) {
    if (ex(d) == 1 && i0 == N - 8) f[xface_at<__half, N>(uint64_t(slot), xdir_index_rt(d), jk)] = uint16_t(q[d][3] >> 16);
    if (ex(d) == -1 && i0 == 0) f[xface_at<__half, N>(uint64_t(slot), xdir_index_rt(d), jk)] = uint16_t(q[d][0] & 0xFFFFu);
  }
}

// ---- layout conversions ------------------------------------------------------

template <typename S>
__global__ void inplace_swap_kernel(S* __restrict__ buf, int64_t ncells, int64_t n3) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ncells) return;
#pragma unroll
  for (int a = 1; a < 19; a += 2) {
    S* p = buf + pdf_at_rt(a, uint64_t(i), uint64_t(n3));
    S* q = buf + pdf_at_rt(a + 1, uint64_t(i), uint64_t(n3));
    const S t = *p;
    *p = *q;
    *q = t;
  }
}

template <typename S>
__global__ void inplace_pair_swap_kernel(S* __restrict__ buf, const int32_t* __restrict__ nbr, int64_t ncells, int n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ncells) return;
  const int64_t n3 = int64_t(n) * n * n;
  const int64_t slot = i / n3;
  const int cell = int(i - slot * n3);
  const int x = cell % n, y = (cell / n) % n, z = cell / (n * n);
  auto side = [n](int c) { return c < 0 ? -1 : (c >= n ? 1 : 0); };
  for (int a = 1; a < 19; a += 2) {
    const int sx = x - ex(a), sy = y - ey(a), sz = z - ez(a);
    const int nb = nbr[slot * 27 + 13 + side(sx) + 3 * side(sy) + 9 * side(sz)];
    if (nb < 0) continue;  // wall: the location keeps its value
    const int sc = ((sx + n) % n) + n * (((sy + n) % n) + n * ((sz + n) % n));
    S* p = buf + pdf_at_rt(a, uint64_t(i), uint64_t(n3));
    S* q = buf + pdf_at_rt(opp(a), uint64_t(nb) * uint64_t(n3) + uint64_t(sc), uint64_t(n3));
    const S t = *p;
    *p = *q;
    *q = t;
  }
}

// Entry buffer -> buffer: the values that entered through x faces, back
// into their places (before the pushed layout is converted).
template <typename S>
__global__ void inplace_entry_merge_kernel(S* __restrict__ buf, const S* __restrict__ entry, int64_t count, int n) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int64_t n2 = int64_t(n) * n;
  int64_t slot, jk;
  int q;
  xface_decode<S>(e, n, slot, q, jk);
  const int a = xdir_dir(q);
  const int x = ex(a) > 0 ? 0 : n - 1;
  buf[pdf_at_rt(a, uint64_t(slot) * uint64_t(n2 * n) + uint64_t(x + n * jk), uint64_t(n2 * n))] = entry[e];
}

// Saves of the state at the start of a parent step from the natural layout:
// every value whose destination lies in the coarser region.
template <typename S, int N>
__global__ void inplace_save_fill_kernel(const S* __restrict__ buf, S* __restrict__ save, const int32_t* __restrict__ nbr,
                                         int64_t ncells) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ncells) return;
  constexpr int64_t N3 = int64_t(N) * N * N;
  const int64_t slot = e / N3;
  const int cell = int(e - slot * N3);
  const int x = cell % N, y = (cell / N) % N, z = cell / (N * N);
  auto side = [](int c) { return c < 0 ? -1 : (c >= N ? 1 : 0); };
  for (int a = 1; a < 19; ++a) {
    const int code = nbr[slot * 27 + 13 + side(x + ex(a)) + 3 * side(y + ey(a)) + 9 * side(z + ez(a))];
    if (code <= kNbrCoarse0) save[save_index<N>(uint32_t(slot), a, x, y, z)] = buf[pdf_index<N>(a, uint64_t(slot), uint32_t(cell))];
  }
}

template <typename S>
int64_t inplace_grid_t(int n, int64_t nblocks) {
  switch (n) {
    case 4: return nblocks * IGeo<S, 4>::TPB;
    case 8: return nblocks * IGeo<S, 8>::TPB;
    case 16: return nblocks * IGeo<S, 16>::TPB;
    case 32: return nblocks * IGeo<S, 32>::TPB;
    default: return -1;
  }
}

template <typename S>
hipError_t launch_inplace_t(int n, const InplaceArgs& a, bool odd, hipStream_t stream) {
  auto go = [&](auto nn) -> hipError_t {
    constexpr int N = decltype(nn)::value;
    const int64_t grid = int64_t(a.nblocks) * IGeo<S, N>::TPB;
    if (grid <= 0) return hipSuccess;
    if (grid > int64_t(0x7FFFFFFF)) return hipErrorInvalidValue;
    const dim3 g = dim3(unsigned(grid)), t = dim3(unsigned(IGeo<S, N>::T));
    if constexpr (IGeo<S, N>::PACKED) {
      auto go8 = [&](auto trt, auto ref) {
        constexpr bool TRT = decltype(trt)::value, REF = decltype(ref)::value;
        if (odd)
          hipLaunchKernelGGL((inplace_odd_h8_kernel<N, TRT, REF>), g, t, 0, stream, a);
        else
          hipLaunchKernelGGL((inplace_even_h8_kernel<N, TRT, REF>), g, t, 0, stream, a);
      };
      using F0 = std::false_type;
      using F1 = std::true_type;
      if (a.refined) {
        if (a.trt)
          go8(F1{}, F1{});
        else
          go8(F0{}, F1{});
      } else {
        if (a.trt)
          go8(F1{}, F0{});
        else
          go8(F0{}, F0{});
      }
      return hipGetLastError();
    } else {
      auto go2 = [&](auto trt, auto ref) {
        constexpr bool TRT = decltype(trt)::value, REF = decltype(ref)::value;
        if (odd)
          hipLaunchKernelGGL((inplace_odd_kernel<S, N, TRT, REF>), g, t, 0, stream, a);
        else
          hipLaunchKernelGGL((inplace_even_kernel<S, N, TRT, REF>), g, t, 0, stream, a);
      };
      using T0 = std::false_type;
      using T1 = std::true_type;
      if (a.refined) {
        if (a.trt)
          go2(T1{}, T1{});
        else
          go2(T0{}, T1{});
      } else {
        if (a.trt)
          go2(T1{}, T0{});
        else
          go2(T0{}, T0{});
      }
      return hipGetLastError();
    }
  };
  switch (n) {
    case 4: return go(std::integral_constant<int, 4>{});
    case 8: return go(std::integral_constant<int, 8>{});
    case 16: return go(std::integral_constant<int, 16>{});
    case 32: return go(std::integral_constant<int, 32>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dev

int64_t inplace_grid(int storage, int n, int64_t nblocks) {
  switch (storage) {
    case 0: return dev::inplace_grid_t<double>(n, nblocks);
    case 1: return dev::inplace_grid_t<float>(n, nblocks);
    case 2: return dev::inplace_grid_t<__half>(n, nblocks);
    default: return -1;
  }
}

hipError_t launch_inplace(int storage, int n, const InplaceArgs& a, bool odd, hipStream_t stream) {
  if (!a.buf || !a.face || !a.entry || !a.nbr) return hipErrorInvalidValue;
  if (a.refined && (!a.flags || !a.par || !a.par_face || !a.save_in || !a.save_out || !a.err)) return hipErrorInvalidValue;
  switch (storage) {
    case 0: return dev::launch_inplace_t<double>(n, a, odd, stream);
    case 1: return dev::launch_inplace_t<float>(n, a, odd, stream);
    case 2: return dev::launch_inplace_t<__half>(n, a, odd, stream);
    default: return hipErrorInvalidValue;
  }
}

namespace {
constexpr int kConvThreads = 256;
template <typename F>
hipError_t by_storage(int storage, F&& f) {
  switch (storage) {
    case 0: return f(double{});
    case 1: return f(float{});
    case 2: return f(__half{});
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t launch_inplace_swap(int storage, int n, void* buf, int64_t nblocks, hipStream_t stream) {
  const int64_t n3 = int64_t(n) * n * n, ncells = nblocks * n3;
  if (ncells <= 0) return hipSuccess;
  const unsigned grid = unsigned((ncells + kConvThreads - 1) / kConvThreads);
  return by_storage(storage, [&](auto s) -> hipError_t {
    using S = decltype(s);
    hipLaunchKernelGGL(dev::inplace_swap_kernel<S>, dim3(grid), dim3(kConvThreads), 0, stream, static_cast<S*>(buf),
                       ncells, n3);
    return hipGetLastError();
  });
}

hipError_t launch_inplace_save_fill(int storage, int n, const void* buf, void* save, const int32_t* nbr, int64_t nblocks,
                                    hipStream_t stream) {
  const int64_t ncells = nblocks * int64_t(n) * n * n;
  if (ncells <= 0) return hipSuccess;
  const unsigned grid = unsigned((ncells + kConvThreads - 1) / kConvThreads);
  return by_storage(storage, [&](auto s) -> hipError_t {
    using S = decltype(s);
    auto go = [&](auto nn) -> hipError_t {
      constexpr int N = decltype(nn)::value;
      hipLaunchKernelGGL((dev::inplace_save_fill_kernel<S, N>), dim3(grid), dim3(kConvThreads), 0, stream,
                         static_cast<const S*>(buf), static_cast<S*>(save), nbr, ncells);
      return hipGetLastError();
    };
    switch (n) {
      case 4: return go(std::integral_constant<int, 4>{});
      case 8: return go(std::integral_constant<int, 8>{});
      case 16: return go(std::integral_constant<int, 16>{});
      case 32: return go(std::integral_constant<int, 32>{});
      default: return hipErrorInvalidValue;
    }
  });
}

hipError_t launch_inplace_entry_merge(int storage, int n, void* buf, const void* entry, int64_t nblocks,
                                      hipStream_t stream) {
  const int64_t count = nblocks * dev::kXDirs * int64_t(n) * n;
  if (count <= 0) return hipSuccess;
  const unsigned grid = unsigned((count + kConvThreads - 1) / kConvThreads);
  return by_storage(storage, [&](auto s) -> hipError_t {
    using S = decltype(s);
    hipLaunchKernelGGL(dev::inplace_entry_merge_kernel<S>, dim3(grid), dim3(kConvThreads), 0, stream,
                       static_cast<S*>(buf), static_cast<const S*>(entry), count, n);
    return hipGetLastError();
  });
}

hipError_t launch_inplace_pair_swap(int storage, int n, void* buf, const int32_t* nbr, int64_t nblocks,
                                    hipStream_t stream) {
  const int64_t ncells = nblocks * int64_t(n) * n * n;
  if (ncells <= 0) return hipSuccess;
  const unsigned grid = unsigned((ncells + kConvThreads - 1) / kConvThreads);
  return by_storage(storage, [&](auto s) -> hipError_t {
    using S = decltype(s);
    hipLaunchKernelGGL(dev::inplace_pair_swap_kernel<S>, dim3(grid), dim3(kConvThreads), 0, stream,
                       static_cast<S*>(buf), nbr, ncells, n);
    return hipGetLastError();
  });
}

}  // namespace lbm
