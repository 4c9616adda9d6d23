// HIP helper kernels of the library (initial state, moments, raw PDF I/O,
// FP64 reductions) and the storage dispatch of the sweep.  PDF buffers are
// block-major: element (a, slot, cell) at (19 slot + a) n^3 + cell; interior
// cells of a level are addressed by their canonical index slot * n^3 + cell.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "forest.hpp"
#include "inplace_save.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

namespace lbm {

hipError_t launch_sweep_f64(int n, const SweepArgs& a, int grid, int split, hipStream_t stream);
hipError_t launch_sweep_f32(int n, const SweepArgs& a, int grid, int split, hipStream_t stream);
hipError_t launch_sweep_f16(int n, const SweepArgs& a, int grid, int split, hipStream_t stream);
int sweep_split_f64(int n, int requested);
int sweep_split_f32(int n, int requested);
int sweep_split_f16(int n, int requested);

namespace {
using namespace dev;

// ---- init / moments / raw I/O / reductions -------------------------------

template <typename S, int N>
__global__ void init_kernel(S* buf, const double* rho, const double* u, int64_t ncells, Accel acc) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
  const double r = rho[idx], ux = u[3 * idx], uy = u[3 * idx + 1], uz = u[3 * idx + 2];
  const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    const double eu = ex(a) * ux + ey(a) * uy + ez(a) * uz;
    const double ea = ex(a) * acc.a[0] + ey(a) * acc.a[1] + ez(a) * acc.a[2];
    const double h = wgt<double>(a) * ((r - 1.0) + 3.0 * eu + 4.5 * eu * eu - usq) + 3.0 * wgt<double>(a) * ea;
    Form<S>::st(buf + pdf_at<N>(a, idx), typename Form<S>::C(h));
  }
}

// Cells [first, first + count) of a level; output index relative to first.
template <typename S, int N>
__global__ void moments_kernel(const S* buf, double* rho, double* u, int64_t first, int64_t count, Accel acc) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int64_t idx = first + t;
  double s = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    const double h = double(Form<S>::ld(buf + pdf_at<N>(a, idx)));
    s += h;
    jx += ex(a) * h;
    jy += ey(a) * h;
    jz += ez(a) * h;
  }
  rho[t] = 1.0 + s;
  u[3 * t] = jx - 0.5 * acc.a[0];
  u[3 * t + 1] = jy - 0.5 * acc.a[1];
  u[3 * t + 2] = jz - 0.5 * acc.a[2];
}

template <typename S, int N>
__global__ void get_pdfs_kernel(const S* buf, double* h, int64_t ncells) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
#pragma unroll
  for (int a = 0; a < 19; ++a) h[idx * 19 + a] = double(Form<S>::ld(buf + pdf_at<N>(a, idx)));
}

template <typename S, int N>
__global__ void set_pdfs_kernel(S* buf, const double* h, int64_t ncells) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
#pragma unroll
  for (int a = 0; a < 19; ++a)
    Form<S>::st(buf + pdf_at<N>(a, idx), typename Form<S>::C(h[idx * 19 + a]));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int kReduceThreads = 256;

// Deterministic FP64 partial sums: fixed grid, fixed per-thread stride,
// wavefront butterfly, then a fixed-order sum over the 4 wavefronts.
template <typename S, int N>
__global__ void __launch_bounds__(kReduceThreads) reduce_kernel(const S* buf, int64_t ncells,
                                                                double* out) {
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < ncells;
       idx += int64_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      const double h = double(Form<S>::ld(buf + pdf_at<N>(a, idx)));
      acc[0] += h;
      acc[1] += ex(a) * h;
      acc[2] += ey(a) * h;
      acc[3] += ez(a) * h;
      acc[4] += (h - h != 0.0) ? 1.0 : 0.0;  // NaN or Inf
    }
  }
  __shared__ double part[kReduceThreads / 64][5];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) part[wv][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double v = 0;
    for (int q = 0; q < kReduceThreads / 64; ++q) v += part[q][threadIdx.x];
    out[blockIdx.x * 5 + threadIdx.x] = v;
  }
}

template <typename S, int N>
__global__ void remap_kernel(RemapArgs a) {
  using C = typename Form<S>::C;
  constexpr int N3 = N * N * N, H = N / 2;
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= a.ncells) return;
  const int64_t b = idx / N3;
  const int local = int(idx - b * N3);
  const int i = local % N, j = (local / N) % N, k = local / (N * N);
  const RemapBlock rb = a.blocks[b];
  C h[19];
  if (rb.mode == 0 || rb.mode == 1) {
    const int src = rb.mode == 0 ? local
                                 : (rb.off[0] + (i >> rb.shift)) + N * ((rb.off[1] + (j >> rb.shift)) +
                                                                       N * (rb.off[2] + (k >> rb.shift)));
    const S* p = static_cast<const S*>(rb.mode == 0 ? a.old_cur[rb.src_level] : a.old_post[rb.src_level]);
#pragma unroll
    for (int d = 0; d < 19; ++d) h[d] = Form<S>::ld(p + pdf_index<N>(d, uint32_t(rb.slot[0]), uint32_t(src)));
  } else {
    const int oct = (i >= H ? 1 : 0) | (j >= H ? 2 : 0) | (k >= H ? 4 : 0);
    const int cx = 2 * (i & (H - 1)), cy = 2 * (j & (H - 1)), cz = 2 * (k & (H - 1));
    const S* p = static_cast<const S*>(a.old_post[rb.src_level]);
#pragma unroll
    for (int d = 0; d < 19; ++d) {
      C s = C(0);
      for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
          for (int ox = 0; ox < 2; ++ox) s += Form<S>::ld(p + pdf_index<N>(d, uint32_t(rb.slot[oct]), (cx + ox) + N * ((cy + oy) + N * (cz + oz))));
      h[d] = s * C(0.125);
    }
  }
  if (rb.mode != 0 && a.collide) {
    // SRT collision in shifted form, as in the sweep
    const C om = sizeof(C) == 8 ? C(a.omega64) : C(a.omega);
    C drho = 0, ux = 0, uy = 0, uz = 0;
#pragma unroll
    for (int d = 0; d < 19; ++d) {
      drho += h[d];
      ux += C(ex(d)) * h[d];
      uy += C(ey(d)) * h[d];
      uz += C(ez(d)) * h[d];
    }
    const C usq = C(1.5) * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int d = 0; d < 19; ++d) {
      const C eu = C(ex(d)) * ux + C(ey(d)) * uy + C(ez(d)) * uz;
      const C heq = wgt<C>(d) * (drho + C(3) * eu + C(4.5) * eu * eu - usq);
      h[d] = h[d] + om * (heq - h[d]);
    }
  }
  S* out = static_cast<S*>(a.dst);
#pragma unroll
  for (int d = 0; d < 19; ++d) Form<S>::st(out + pdf_at<N>(d, idx), h[d]);
}

// Neighbour offset (-1, 0, +1) of a local coordinate after a shift.
template <int N>
__device__ __forceinline__ int nb_side(int c) {
  return c < 0 ? -1 : (c >= N ? 1 : 0);
}

// Coalesced pairs (X, a) of one chunk of one fine_nbr row per workgroup,
// the row's neighbour tables in LDS: the mean over the 8 children c of X of
// what the finer level's second stream pulled into c from c - e_a -- the
// fine state after its first substep if c - e_a is a level-(L+1) cell, else
// (c - e_a a halo cell, filled from c - 2 e_a in the first substep) the fine
// state at the start of the parent step if c - 2 e_a is a level-(L+1) cell,
// else the exploded coarse value, which is X's own source value at X - e_a
// (eq. ftoc, Algorithm 1).  Children are summed in (z, y, x) order.
constexpr int kCoalThreads = 256;
static_assert(kCoalThreads * kCoalPairs == kCoalChunk, "coalescence chunk = threads x pairs per thread");

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
        p = xcopy && lx == xout ? static_cast<const S*>(c.fine1_x) + xface_index_rt<N>(A, uint32_t(fy), uint32_t(jk))
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
        p = xcopy && lx == xout ? static_cast<const S*>(c.fine0_x) + xface_index_rt<N>(A, uint32_t(fz), uint32_t(jk))
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

// Coalescence launch: one chunk of at most kCoalThreads * kCoalPairs pairs
// of one coarse block per workgroup, kCoalPairs pairs per thread.  The
// chunk record names the block and its fine_nbr row, so the pair words and
// the block's tables (staged in LDS) are loaded together, and after the
// barrier all source values of a thread are one more memory round trip.
// Children are summed in (z, y, x) order.  Walls and the interpolated
// explosion each have a variant of their own, so the periodic form with the
// homogeneous explosion carries no code for them.
template <typename S, int N, bool INTERP, bool WALLS>
__global__ void __launch_bounds__(kCoalThreads) coalesce_kernel(CoalArgs c) {
  using C = typename Form<S>::C;
  constexpr int P = kCoalPairs;
  __shared__ int32_t fns[8 * 27];
  __shared__ int32_t nbs[27];
  const int row = c.chunks[4 * blockIdx.x], slot = c.chunks[4 * blockIdx.x + 1];
  const int first = c.chunks[4 * blockIdx.x + 2], end = c.chunks[4 * blockIdx.x + 3];
  uint32_t w[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int t = first + int(threadIdx.x) + p * kCoalThreads;
    w[p] = t < end ? c.pairs[t] : 0xFFFFFFFFu;
  }
  for (int q = threadIdx.x; q < 8 * 27; q += blockDim.x) fns[q] = c.fine_nbr[int64_t(row) * 216 + q];
  for (int q = threadIdx.x; q < 27; q += blockDim.x) nbs[q] = c.nbr[int64_t(slot) * 27 + q];
  __syncthreads();
  const S* ptr[P][8];
  bool own[P][8];
  C iv[P][8];
  bool use_iv[P][8];
  const S* rp[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const bool valid = w[p] != 0xFFFFFFFFu;
    pair_sources<S, N, INTERP, WALLS>(c, fns, nbs, valid ? int(w[p] >> 16) : 0, valid ? int(w[p] & 0xFFFFu) : 0, ptr[p], own[p],
                       iv[p], use_iv[p], rp[p]);
  }
  C v[P][8], regular[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[p][q] = INTERP && use_iv[p][q] ? iv[p][q] : C(Form<S>::ld(ptr[p][q]));
    regular[p] = C(Form<S>::ld(rp[p]));
  }
  CheckAcc acc;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (w[p] == 0xFFFFFFFFu) continue;
    const int A = int(w[p] >> 16), cell = int(w[p] & 0xFFFFu);
    const int i = cell % N, j = (cell / N) % N, k = cell / (N * N);
    C sum = C(0);
#pragma unroll
    for (int q = 0; q < 8; ++q) sum += own[p][q] ? v[p][q] : regular[p];
    if (c.check) check_sum<C>(acc, v[p], own[p], regular[p], sum);
    // a pair entering through an x face goes to the x-face layout
    const int EX = ex(A);
    S* o = EX != 0 && i == (EX > 0 ? 0 : N - 1)
               ? static_cast<S*>(c.out_x) + xface_index_rt<N>(A, uint32_t(row), uint32_t(j + N * k))
               : static_cast<S*>(c.out) + pdf_index<N>(A, uint32_t(row), uint32_t(cell));
    Form<S>::st(o, sum * C(0.125));
  }
  if (c.check) check_flush(c.check, acc);
}

// x-face copy of a buffer (see CoalArgs): one thread per element of xf.
template <typename S, int N>
__global__ void face_copy_kernel(const S* buf, S* xf, int64_t count) {
  constexpr int N2 = N * N;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int64_t slot = e / (kXDirs * N2);
  const int A = xdir_dir(int((e / N2) % kXDirs));
  const int jk = int(e % N2);
  xf[e] = buf[pdf_index<N>(A, uint64_t(slot), uint32_t((ex(A) < 0 ? 0 : N - 1) + N * jk))];
}

template <typename F>
hipError_t dispatch(int storage, int n, F&& f) {
  auto by_n = [&](auto tag) -> hipError_t {
    using S = decltype(tag);
    switch (n) {
      case 4: return f(S{}, std::integral_constant<int, 4>{});
      case 8: return f(S{}, std::integral_constant<int, 8>{});
      case 16: return f(S{}, std::integral_constant<int, 16>{});
      case 32: return f(S{}, std::integral_constant<int, 32>{});
      default: return hipErrorInvalidValue;
    }
  };
  switch (storage) {
    case 0: return by_n(double{});
    case 1: return by_n(float{});
    case 2: return by_n(__half{});
    default: return hipErrorInvalidValue;
  }
}

inline unsigned grid_for(int64_t n, int threads) { return unsigned((n + threads - 1) / threads); }

}  // namespace

int sweep_tile_cells(int storage, int n) {
  const int n3 = n * n * n;
  const int w = storage == 0 ? Vec<double>::W : (storage == 2 && n >= 8 ? 8 : Vec<float>::W);
  return n3 < 256 * w ? n3 : 256 * w;
}

int sweep_split(int storage, int n, int requested) {
  switch (storage) {
    case 0: return sweep_split_f64(n, requested);
    case 1: return sweep_split_f32(n, requested);
    case 2: return sweep_split_f16(n, requested);
    default: return 1;
  }
}

hipError_t launch_sweep(int storage, int n, const SweepArgs& a, int grid, int split, hipStream_t stream) {
  if (a.nwork <= 0) return hipSuccess;
  switch (storage) {
    case 0: return launch_sweep_f64(n, a, grid, split, stream);
    case 1: return launch_sweep_f32(n, a, grid, split, stream);
    case 2: return launch_sweep_f16(n, a, grid, split, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init(int storage, int n, void* buf, const double* rho, const double* u,
                       int64_t ncells, Accel accel, hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((init_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream, static_cast<S*>(buf),
                       rho, u, ncells, accel);
    return hipGetLastError();
  });
}

hipError_t launch_moments(int storage, int n, const void* buf, double* rho, double* u, int64_t first,
                          int64_t count, Accel accel, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((moments_kernel<S, N>), dim3(grid_for(count, 256)), dim3(256), 0, stream,
                       static_cast<const S*>(buf), rho, u, first, count, accel);
    return hipGetLastError();
  });
}

hipError_t launch_get_pdfs(int storage, int n, const void* buf, double* h, int64_t ncells,
                           hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((get_pdfs_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream,
                       static_cast<const S*>(buf), h, ncells);
    return hipGetLastError();
  });
}

hipError_t launch_set_pdfs(int storage, int n, void* buf, const double* h, int64_t ncells,
                           hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((set_pdfs_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream,
                       static_cast<S*>(buf), h, ncells);
    return hipGetLastError();
  });
}

hipError_t launch_remap(int storage, int n, const RemapArgs& a, hipStream_t stream) {
  if (a.ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((remap_kernel<S, N>), dim3(grid_for(a.ncells, 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
  });
}

hipError_t launch_coalesce(int storage, int n, const CoalArgs& a, hipStream_t stream) {
  if (a.nchunks <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    // the interpolated explosion and walls each have their own variant, so
    // that the plain periodic form carries no code for them
    if (a.interp && a.walls)
      hipLaunchKernelGGL((coalesce_kernel<S, N, true, true>), dim3(a.nchunks), dim3(kCoalThreads), 0, stream, a);
    else if (a.interp)
      hipLaunchKernelGGL((coalesce_kernel<S, N, true, false>), dim3(a.nchunks), dim3(kCoalThreads), 0, stream, a);
    else if (a.walls)
      hipLaunchKernelGGL((coalesce_kernel<S, N, false, true>), dim3(a.nchunks), dim3(kCoalThreads), 0, stream, a);
    else
      hipLaunchKernelGGL((coalesce_kernel<S, N, false, false>), dim3(a.nchunks), dim3(kCoalThreads), 0, stream, a);
    return hipGetLastError();
  });
}

hipError_t launch_face_copy(int storage, int n, const void* buf, void* xf, int64_t nblocks, hipStream_t stream) {
  if (nblocks <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    const int64_t count = nblocks * kXDirs * N * N;
    hipLaunchKernelGGL((face_copy_kernel<S, N>), dim3(grid_for(count, 256)), dim3(256), 0, stream,
                       static_cast<const S*>(buf), static_cast<S*>(xf), count);
    return hipGetLastError();
  });
}

hipError_t launch_reduce(int storage, int n, const void* buf, int64_t ncells, double* out,
                         hipStream_t stream) {
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((reduce_kernel<S, N>), dim3(kReduceGrid), dim3(kReduceThreads), 0, stream,
                       static_cast<const S*>(buf), ncells, out);
    return hipGetLastError();
  });
}

}  // namespace lbm
