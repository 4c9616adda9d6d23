// Coalescence of one level (eq. ftoc, section 4.4): device code shared by
// the coalescence launch (kernels.hip) and the sweep launch that runs it
// alongside the finer level's second substep (sweep.hpp).
//
// A coalesced pair (X, a), X a level-L cell next to the finer region, gets
// the mean over the 8 children c of X of what the finer level's second
// stream pulled into c from c - e_a: the fine state after its first substep
// if c - e_a is a level-(L+1) cell, else (c - e_a a halo cell, filled from
// c - 2 e_a in the first substep) the fine state at the start of the parent
// step if c - 2 e_a is a level-(L+1) cell, else the exploded coarse value,
// which is X's own source value at X - e_a (eq. ftoc, Algorithm 1).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "forest.hpp"
#include "inplace_save.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

namespace lbm {
namespace dev {

// Neighbour offset (-1, 0, +1) of a local coordinate after a shift.
template <int N>
__device__ __forceinline__ int nb_side(int c) {
  return c < 0 ? -1 : (c >= N ? 1 : 0);
}

// floor(d / 2) for d >= -1
__device__ __forceinline__ int half_floor(int d) { return d < 0 ? -1 : d >> 1; }

// Address of direction a of level-L cell (px, py, pz): local coordinates of
// the coarse block whose table is nbs (entry 13 is the block itself), at
// most one cell beyond it (then the neighbour block from the table, which
// must be a level-L block: a child's two-substep back-trace stays within the
// coarse cells next to X).
template <typename S, int N>
__device__ __forceinline__ const S* coarse_cell(const CoalArgs& c, const int32_t* nbs, int px, int py, int pz, int a) {
  const int nb = nbs[13 + nb_side<N>(px) + 3 * nb_side<N>(py) + 9 * nb_side<N>(pz)];
  if (nb < 0) {
    atomicOr(c.err, kErrNoSource);
    return static_cast<const S*>(c.cur);
  }
  return static_cast<const S*>(c.cur) +
         pdf_index<N>(a, uint32_t(nb), uint32_t((px & (N - 1)) + N * ((py & (N - 1)) + N * (pz & (N - 1)))));
}

// Accumulation check of one coalesced pair (see CoalArgs::check): the same
// 8 values summed in FP64, compared with the compute-type sum.  Recursive
// summation of 8 terms in a type of unit roundoff u errs by at most
// gamma_7 sum |v|, gamma_7 = 7u / (1 - 7u) (Higham, Accuracy and Stability
// of Numerical Algorithms, 2002, eq. (4.4)); the ratio to that bound must
// not exceed 1.
struct CheckAcc {
  double dev = 0.0, ratio = 0.0, count = 0.0;
};
template <typename C>
__device__ __forceinline__ void check_sum(CheckAcc& acc, const C* v, const bool* fine, C regular, C sum) {
  double s = 0.0, a = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double x = double(fine[q] ? v[q] : regular);
    s += x;
    a += fabs(x);
  }
  const double u = sizeof(C) == 8 ? 0x1p-53 : 0x1p-24;
  const double gamma7 = 7.0 * u / (1.0 - 7.0 * u);
  const double dev = fabs(double(sum) - s);
  acc.dev = fmax(acc.dev, 0.125 * dev);
  acc.ratio = fmax(acc.ratio, a > 0.0 ? dev / (gamma7 * a) : 0.0);
  acc.count += 1.0;
}
// Wavefront reduction of the per-lane figures, then one set of atomics per
// wavefront (non-negative doubles order like their bit patterns, so the
// maxima are kept with integer atomics).  Every lane of the wave calls it.
__device__ __forceinline__ void check_flush(unsigned long long* out, CheckAcc acc) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc.dev = fmax(acc.dev, __shfl_xor(acc.dev, off, 64));
    acc.ratio = fmax(acc.ratio, __shfl_xor(acc.ratio, off, 64));
    acc.count += __shfl_xor(acc.count, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(acc.dev));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(acc.ratio));
    atomicAdd(out + 2, (unsigned long long)acc.count);
  }
}

// Sources of one coalesced pair (X, A), X = cell of the chunk's coarse block
// (its table nbs) with the virtual fine blocks of its octants (fns): for each
// of the 8 children c (in (z, y, x) order), what the finer level's second
// stream pulled into c -- from c - e_A after the first substep if that is a
// fine cell; if c - e_A is a wall, c's own bounced-back value of the opposite
// direction Ab after the first substep, pulled from c + e_A at t (fine, or
// the exploded value of its parent); from c - 2 e_A at t if that is a fine
// cell (c - e_A a ghost cell); the ghost cell c - e_A's bounced-back exploded
// value of Ab if c - 2 e_A is a wall; else the exploded value of c - 2 e_A,
// whose parent is X - e_A: X's regular source.  Without interpolation every
// exploded value is its parent's (eq. ctof) and comes as an address in ptr
// (own[q] = false: the regular source); with it, exploded values are
// reconstructed (interp_value) and returned in iv (use_iv[q]).
template <typename S, int N, bool INTERP, bool WALLS>
__device__ __forceinline__ void pair_sources(const CoalArgs& c, const int32_t* fns, const int32_t* nbs, int A, int cell,
                                             const S** ptr, bool* own, typename Form<S>::C* iv, bool* use_iv,
                                             const S*& rp) {
  constexpr int H = N / 2;
  const int i = cell % N, j = (cell / N) % N, k = cell / (N * N);
  const int EX = ex(A), EY = ey(A), EZ = ez(A), Ab = opp(A);
  const int sx = i - EX, sy = j - EY, sz = k - EZ;
  const int nb = nbs[13 + nb_side<N>(sx) + 3 * nb_side<N>(sy) + 9 * nb_side<N>(sz)];
  rp = static_cast<const S*>(c.cur) +
       (nb >= 0 ? pdf_index<N>(A, uint32_t(nb), uint32_t((sx & (N - 1)) + N * ((sy & (N - 1)) + N * (sz & (N - 1))))) : 0);
  const int oct = (i >= H ? 1 : 0) | (j >= H ? 2 : 0) | (k >= H ? 4 : 0);
  const int32_t* fn = fns + oct * 27;
  const int cx = 2 * (i & (H - 1)), cy = 2 * (j & (H - 1)), cz = 2 * (k & (H - 1));
  // a fine value at the x face it leaves through comes from the x-face copy
  const int xout = EX < 0 ? 0 : N - 1;
  const bool xcopy = EX != 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ox = q & 1, oy = (q >> 1) & 1, oz = q >> 2;
    const int yx = cx + ox - EX, yy = cy + oy - EY, yz = cz + oz - EZ;
    const int fy = fn[13 + nb_side<N>(yx) + 3 * nb_side<N>(yy) + 9 * nb_side<N>(yz)];
    const int zx = yx - EX, zy = yy - EY, zz = yz - EZ;
    const int fz = fn[13 + nb_side<N>(zx) + 3 * nb_side<N>(zy) + 9 * nb_side<N>(zz)];
    const S* p = static_cast<const S*>(c.cur);
    bool o = true;
    use_iv[q] = false;
    if (fy >= 0) {
      const int lx = yx & (N - 1), jk = (yy & (N - 1)) + N * (yz & (N - 1));
      if (c.save_half)
        p = static_cast<const S*>(c.save_half) + save_index<N>(uint32_t(fy), A, lx, yy & (N - 1), yz & (N - 1));
      else
        p = xcopy && lx == xout ? static_cast<const S*>(c.fine1_x) + xface_index_rt<S, N>(A, uint32_t(fy), uint32_t(jk))
                                : static_cast<const S*>(c.fine1) + pdf_index<N>(A, uint32_t(fy), uint32_t(lx + N * jk));
    } else if (WALLS && fy == kFineWall) {
      const int wx = cx + ox + EX, wy = cy + oy + EY, wz = cz + oz + EZ;
      const int fw = fn[13 + nb_side<N>(wx) + 3 * nb_side<N>(wy) + 9 * nb_side<N>(wz)];
      if (fw >= 0 && c.save_t) {
        p = static_cast<const S*>(c.save_t) + save_index<N>(uint32_t(fw), Ab, wx & (N - 1), wy & (N - 1), wz & (N - 1));
      } else if (fw >= 0) {
        p = static_cast<const S*>(c.fine0) +
            pdf_index<N>(Ab, uint32_t(fw), uint32_t((wx & (N - 1)) + N * ((wy & (N - 1)) + N * (wz & (N - 1)))));
      } else if (INTERP) {
        iv[q] = interp_value<S, N>(static_cast<const S*>(c.cur), nbs, i + half_floor(ox + EX), j + half_floor(oy + EY),
                                   k + half_floor(oz + EZ), Ab, (ox + EX) & 1, (oy + EY) & 1, (oz + EZ) & 1, c.err);
        use_iv[q] = true;
      } else {
        p = coarse_cell<S, N>(c, nbs, i + half_floor(ox + EX), j + half_floor(oy + EY), k + half_floor(oz + EZ), Ab);
      }
    } else if (fz >= 0) {
      const int lx = zx & (N - 1), jk = (zy & (N - 1)) + N * (zz & (N - 1));
      if (c.save_t)
        p = static_cast<const S*>(c.save_t) + save_index<N>(uint32_t(fz), A, lx, zy & (N - 1), zz & (N - 1));
      else
        p = xcopy && lx == xout ? static_cast<const S*>(c.fine0_x) + xface_index_rt<S, N>(A, uint32_t(fz), uint32_t(jk))
                                : static_cast<const S*>(c.fine0) + pdf_index<N>(A, uint32_t(fz), uint32_t(lx + N * jk));
    } else if (WALLS && fz == kFineWall) {
      if (INTERP) {
        iv[q] = interp_value<S, N>(static_cast<const S*>(c.cur), nbs, i + half_floor(ox - EX), j + half_floor(oy - EY),
                                   k + half_floor(oz - EZ), Ab, (ox - EX) & 1, (oy - EY) & 1, (oz - EZ) & 1, c.err);
        use_iv[q] = true;
      } else {
        p = coarse_cell<S, N>(c, nbs, i + half_floor(ox - EX), j + half_floor(oy - EY), k + half_floor(oz - EZ), Ab);
      }
    } else if (INTERP) {
      // the exploded value of c - 2 e_A inside its parent X - e_A, at the
      // octant of c inside X
      iv[q] = interp_value<S, N>(static_cast<const S*>(c.cur), nbs, sx, sy, sz, A, ox, oy, oz, c.err);
      use_iv[q] = true;
    } else {
      o = false;
    }
    own[q] = o;
    ptr[q] = p;
  }
}

// One chunk of coalesced pairs (at most kCoalChunk of one coarse block and
// one direction; record in CoalArgs::chunks) by the calling workgroup, its
// lanes taking the pairs in turn.  The chunk record names the block, its
// fine_nbr row and the direction, so the direction and everything derived
// from it are uniform over the workgroup; the block's tables are staged in
// LDS (fns: 8 x 27 entries, nbs: 27), after which every source value of a
// pair is one memory round trip.  Lanes past the chunk's end repeat its
// first pair and store nothing.  Children are summed in (z, y, x) order.
// Every lane of the workgroup must call it with the same chunk.
template <typename S, int N, bool INTERP, bool WALLS>
__device__ __forceinline__ void coalesce_chunk(const CoalArgs& c, int chunk, int32_t* fns, int32_t* nbs) {
  using C = typename Form<S>::C;
  const int32_t* rec = c.chunks + 4 * int64_t(chunk);
  const int row = rec[0], slot = rec[1], first = rec[2], cw = rec[3];
  const int count = cw & 0xFFFF, A = cw >> 16;
  if (count == 0) return;  // padding chunk
  for (int q = threadIdx.x; q < 8 * 27; q += blockDim.x) fns[q] = c.fine_nbr[int64_t(row) * 216 + q];
  for (int q = threadIdx.x; q < 27; q += blockDim.x) nbs[q] = c.nbr[int64_t(slot) * 27 + q];
  __syncthreads();
  CheckAcc acc;
  for (int t0 = 0; t0 < count; t0 += int(blockDim.x)) {
    const int t = t0 + int(threadIdx.x);
    const bool valid = t < count;
    const int cell = int(c.cells[first + (valid ? t : 0)]);
    const S* ptr[8];
    bool own[8];
    C iv[8];
    bool use_iv[8];
    const S* rp;
    pair_sources<S, N, INTERP, WALLS>(c, fns, nbs, A, cell, ptr, own, iv, use_iv, rp);
    C v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = INTERP && use_iv[q] ? iv[q] : C(Form<S>::ld(ptr[q]));
    const C regular = C(Form<S>::ld(rp));
    if (valid) {
      const int i = cell % N, j = (cell / N) % N, k = cell / (N * N);
      C sum = C(0);
#pragma unroll
      for (int q = 0; q < 8; ++q) sum += own[q] ? v[q] : regular;
      if (c.check) check_sum<C>(acc, v, own, regular, sum);
      // a pair entering through an x face goes to the x-face layout
      const int EX = ex(A);
      S* o = EX != 0 && i == (EX > 0 ? 0 : N - 1)
                 ? static_cast<S*>(c.out_x) + xface_index_rt<S, N>(A, uint32_t(row), uint32_t(j + N * k))
                 : static_cast<S*>(c.out) + pdf_index<N>(A, uint32_t(row), uint32_t(cell));
      Form<S>::st(o, sum * C(0.125));
    }
  }
  if (c.check) check_flush(c.check, acc);
}

}  // namespace dev
}  // namespace lbm
