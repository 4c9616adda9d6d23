// HIP kernels for gfx950: the fused refined-LBM sweep and its helpers.
//
// One launch of `sweep_kernel` performs one substep of one level L
// (section 4, Algorithm 1, in post-collision form):
//
//   for every live cell x of level L (interior cells of the level-L blocks
//   and the halo cells of its ghost blocks) and every direction a:
//     - (x, a) in the coalescence set  -> mean of the 8 children of x in
//       level L+1 after its two substeps (eq. ftoc);
//     - source x - e_a inside a level-L block -> that block's value;
//     - source in a ghost block (coarser region):
//         substep 1: the parent's post-collision value (explosion eq. ctof,
//                    done as a gather, nothing is written);
//         substep 2: the ghost block's halo value from substep 1 if the
//                    source is a halo cell, else the parent's value;
//   interior cells are then collided (SRT, eq. fequ) and written; halo cells
//   are written uncollided (ghost layers are streamed, never collided).
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
// Memory layout per level: [slot][direction][z][y][x], one slot per block,
// so a 64-lane wavefront reads 64 consecutive cells of one direction.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "forest.hpp"
#include "kernels.hpp"

namespace lbm {
namespace {

// ---- D3Q19 velocity set (rest, 6 faces, 12 edges; opposites adjacent) ----
__host__ __device__ constexpr int ex(int a) {
  return a == 1 || a == 7 || a == 9 || a == 11 || a == 13 ? 1 : (a == 2 || a == 8 || a == 10 || a == 12 || a == 14 ? -1 : 0);
}
__host__ __device__ constexpr int ey(int a) {
  return a == 3 || a == 7 || a == 10 || a == 15 || a == 17 ? 1 : (a == 4 || a == 8 || a == 9 || a == 16 || a == 18 ? -1 : 0);
}
__host__ __device__ constexpr int ez(int a) {
  return a == 5 || a == 11 || a == 14 || a == 15 || a == 18 ? 1 : (a == 6 || a == 12 || a == 13 || a == 16 || a == 17 ? -1 : 0);
}
template <typename C>
__host__ __device__ constexpr C wgt(int a) {
  return a == 0 ? C(1) / C(3) : (a <= 6 ? C(1) / C(18) : C(1) / C(36));
}

// ---- storage forms --------------------------------------------------------
template <typename S>
struct Form;
template <>
struct Form<double> {
  using C = double;
  static __device__ __forceinline__ double ld(const double* p) { return *p; }
  static __device__ __forceinline__ void st(double* p, double v) { *p = v; }
  static __device__ __forceinline__ double omega(const SweepArgs& a) { return a.omega64; }
};
template <>
struct Form<float> {
  using C = float;
  static __device__ __forceinline__ float ld(const float* p) { return *p; }
  static __device__ __forceinline__ void st(float* p, float v) { *p = v; }
  static __device__ __forceinline__ float omega(const SweepArgs& a) { return a.omega; }
};
template <>
struct Form<__half> {
  using C = float;
  static __device__ __forceinline__ float ld(const __half* p) { return __half2float(*p); }
  static __device__ __forceinline__ void st(__half* p, float v) { *p = __float2half_rn(v); }
  static __device__ __forceinline__ float omega(const SweepArgs& a) { return a.omega; }
};

template <int N>
struct Geo {
  static constexpr int N3 = N * N * N;
  static constexpr int T = N3 < 256 ? N3 : 256;  // cells per tile = threads per workgroup
  static constexpr int TPB = N3 / T;             // tiles per block
  static constexpr int H = N / 2;
};

template <int N>
__device__ __forceinline__ int zone_of(int i, int j, int k) {
  auto z = [](int c) { return c < 2 ? 0 : (c >= N - 2 ? 2 : 1); };
  return z(i) + 3 * z(j) + 9 * z(k);
}

template <typename S, int N>
__device__ __forceinline__ const S* pdf_ptr(const S* base, int slot, int a) {
  return base + (size_t(slot) * 19 + a) * Geo<N>::N3;
}

// Coalescence: mean of the 8 children of cell (i, j, k) of real slot `slot`.
template <typename S, int N, int A>
__device__ __forceinline__ typename Form<S>::C coalesce(const SweepArgs& a, int slot, int i, int j, int k) {
  using C = typename Form<S>::C;
  constexpr int H = Geo<N>::H;
  const int oct = (i >= H ? 1 : 0) | (j >= H ? 2 : 0) | (k >= H ? 4 : 0);
  const int cg = a.child_ghost[slot * 8 + oct];
  if (cg < 0) {
    atomicOr(a.err, kErrNoChild);
    return C(0);
  }
  const S* p = pdf_ptr<S, N>(static_cast<const S*>(a.fine), cg, A);
  const int cx = 2 * (i & (H - 1)), cy = 2 * (j & (H - 1)), cz = 2 * (k & (H - 1));
  C s = C(0);
#pragma unroll
  for (int oz = 0; oz < 2; ++oz)
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
      for (int ox = 0; ox < 2; ++ox) s += Form<S>::ld(p + (cx + ox) + N * ((cy + oy) + N * (cz + oz)));
  return s * C(0.125);
}

// Pull of direction A for cell (i, j, k) of slot `slot`.
template <typename S, int N, int A, bool SIMPLE>
__device__ __forceinline__ typename Form<S>::C pull(const SweepArgs& a, const int32_t* snbr, int slot, uint32_t fl,
                                                    int i, int j, int k) {
  using C = typename Form<S>::C;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const int sx = i - EX, sy = j - EY, sz = k - EZ;
  const int ox = EX == 0 ? 0 : (sx < 0 ? -1 : (sx >= N ? 1 : 0));
  const int oy = EY == 0 ? 0 : (sy < 0 ? -1 : (sy >= N ? 1 : 0));
  const int oz = EZ == 0 ? 0 : (sz < 0 ? -1 : (sz >= N ? 1 : 0));
  const int lx = sx & (N - 1), ly = sy & (N - 1), lz = sz & (N - 1);
  const int ls = lx + N * (ly + N * lz);
  const int dir = 13 + ox + 3 * oy + 9 * oz;
  const int nb = dir == 13 ? slot : snbr[dir];
  const S* cur = static_cast<const S*>(a.cur);
  if (SIMPLE) return Form<S>::ld(pdf_ptr<S, N>(cur, nb, A) + ls);

  if (fl & kHasFine) {
    // (x, A) is coalesced if x - e_A, or for an edge direction one of its two
    // axis projections, lies in region(L+1)
    bool coal = dir != 13 && nb == kNbrFine;
    if (A >= 7) {
      // neighbour directions of the two axis projections of x - e_A
      const int dA = EX != 0 ? 13 + ox : 13 + 3 * oy;
      const int dB = EZ != 0 ? 13 + 9 * oz : 13 + 3 * oy;
      coal = coal || (dA != 13 && snbr[dA] == kNbrFine) || (dB != 13 && snbr[dB] == kNbrFine);
    }
    if (coal) return coalesce<S, N, A>(a, slot, i, j, k);
  }
  if (nb >= 0 && nb < a.nreal) return Form<S>::ld(pdf_ptr<S, N>(cur, nb, A) + ls);
  if (nb < 0) {
    atomicOr(a.err, kErrNoSource);
    return C(0);
  }
  // source in a ghost block
  if (a.substep == 2 && ((a.zmask[nb] >> zone_of<N>(lx, ly, lz)) & 1u))
    return Form<S>::ld(pdf_ptr<S, N>(cur, nb, A) + ls);
  const int pp = a.parent[nb];
  const int oc = pp & 7;
  constexpr int H = Geo<N>::H;
  const int px = (oc & 1 ? H : 0) + (lx >> 1), py = (oc & 2 ? H : 0) + (ly >> 1), pz = (oc & 4 ? H : 0) + (lz >> 1);
  return Form<S>::ld(pdf_ptr<S, N>(static_cast<const S*>(a.par), pp >> 3, A) + px + N * (py + N * pz));
}

template <typename S, int N, bool SIMPLE, int A = 0>
__device__ __forceinline__ void pull_all(const SweepArgs& a, const int32_t* snbr, int slot, uint32_t fl, int i, int j,
                                         int k, typename Form<S>::C* h) {
  h[A] = pull<S, N, A, SIMPLE>(a, snbr, slot, fl, i, j, k);
  if constexpr (A + 1 < 19) pull_all<S, N, SIMPLE, A + 1>(a, snbr, slot, fl, i, j, k, h);
}

template <typename C, int A = 0>
__device__ __forceinline__ void relax(C* h, C drho, C ux, C uy, C uz, C usq, C om) {
  constexpr C w = wgt<C>(A);
  const C eu = C(ex(A)) * ux + C(ey(A)) * uy + C(ez(A)) * uz;
  const C heq = w * (drho + C(3) * eu + C(4.5) * eu * eu - usq);
  h[A] = h[A] + om * (heq - h[A]);
  if constexpr (A + 1 < 19) relax<C, A + 1>(h, drho, ux, uy, uz, usq, om);
}

// SRT collision in shifted form (rho0 = 1).
template <typename C>
__device__ __forceinline__ void collide(C* h, C om) {
  C drho = C(0), ux = C(0), uy = C(0), uz = C(0);
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    drho += h[a];
    if (ex(a)) ux += ex(a) > 0 ? h[a] : -h[a];
    if (ey(a)) uy += ey(a) > 0 ? h[a] : -h[a];
    if (ez(a)) uz += ez(a) > 0 ? h[a] : -h[a];
  }
  const C usq = C(1.5) * (ux * ux + uy * uy + uz * uz);
  relax<C>(h, drho, ux, uy, uz, usq, om);
}

template <typename S, int N>
__global__ void __launch_bounds__(Geo<N>::T) sweep_kernel(SweepArgs a) {
  using C = typename Form<S>::C;
  constexpr int T = Geo<N>::T, TPB = Geo<N>::TPB;
  __shared__ int32_t snbr[27];
  const C om = Form<S>::omega(a);
  S* nxt = static_cast<S*>(a.nxt);
  for (int w = blockIdx.x; w < a.nwork; w += gridDim.x) {
    const int item = a.work[w];
    const int slot = item / TPB;
    const int local = (item - slot * TPB) * T + int(threadIdx.x);
    __syncthreads();
    if (threadIdx.x < 27) snbr[threadIdx.x] = a.nbr[slot * 27 + threadIdx.x];
    __syncthreads();
    const uint32_t fl = a.flags[slot];
    const int i = local & (N - 1), j = (local / N) & (N - 1), k = local / (N * N);
    C h[19];
    if (fl & kAllSameLevel) {
      pull_all<S, N, true>(a, snbr, slot, fl, i, j, k, h);
      collide<C>(h, om);
    } else {
      if (!(fl & kReal) && !((a.zmask[slot] >> zone_of<N>(i, j, k)) & 1u)) continue;
      pull_all<S, N, false>(a, snbr, slot, fl, i, j, k, h);
      if (fl & kReal) collide<C>(h, om);
    }
    S* out = nxt + size_t(slot) * 19 * Geo<N>::N3 + local;
#pragma unroll
    for (int d = 0; d < 19; ++d) Form<S>::st(out + size_t(d) * Geo<N>::N3, h[d]);
  }
}

// ---- init / moments / raw I/O / reductions -------------------------------

template <typename S, int N>
__global__ void init_kernel(S* buf, const double* rho, const double* u, int64_t ncells) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
  constexpr int N3 = Geo<N>::N3;
  const int64_t slot = idx / N3;
  const int local = int(idx - slot * N3);
  const double r = rho[idx], ux = u[3 * idx], uy = u[3 * idx + 1], uz = u[3 * idx + 2];
  const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    const double eu = ex(a) * ux + ey(a) * uy + ez(a) * uz;
    const double h = wgt<double>(a) * ((r - 1.0) + 3.0 * eu + 4.5 * eu * eu - usq);
    Form<S>::st(buf + (slot * 19 + a) * N3 + local, typename Form<S>::C(h));
  }
}

template <typename S, int N>
__global__ void moments_kernel(const S* buf, double* rho, double* u, int64_t ncells) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
  constexpr int N3 = Geo<N>::N3;
  const int64_t slot = idx / N3;
  const int local = int(idx - slot * N3);
  double s = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    const double h = double(Form<S>::ld(buf + (slot * 19 + a) * N3 + local));
    s += h;
    jx += ex(a) * h;
    jy += ey(a) * h;
    jz += ez(a) * h;
  }
  rho[idx] = 1.0 + s;
  u[3 * idx] = jx;
  u[3 * idx + 1] = jy;
  u[3 * idx + 2] = jz;
}

template <typename S, int N>
__global__ void get_pdfs_kernel(const S* buf, double* h, int64_t ncells) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
  constexpr int N3 = Geo<N>::N3;
  const int64_t slot = idx / N3;
  const int local = int(idx - slot * N3);
#pragma unroll
  for (int a = 0; a < 19; ++a) h[idx * 19 + a] = double(Form<S>::ld(buf + (slot * 19 + a) * N3 + local));
}

template <typename S, int N>
__global__ void set_pdfs_kernel(S* buf, const double* h, int64_t ncells) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
  constexpr int N3 = Geo<N>::N3;
  const int64_t slot = idx / N3;
  const int local = int(idx - slot * N3);
#pragma unroll
  for (int a = 0; a < 19; ++a)
    Form<S>::st(buf + (slot * 19 + a) * N3 + local, typename Form<S>::C(h[idx * 19 + a]));
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
__global__ void __launch_bounds__(kReduceThreads) reduce_kernel(const S* buf, int64_t ncells, double* out) {
  constexpr int N3 = Geo<N>::N3;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < ncells;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int64_t slot = idx / N3;
    const int local = int(idx - slot * N3);
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      const double h = double(Form<S>::ld(buf + (slot * 19 + a) * N3 + local));
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

hipError_t launch_sweep(int storage, int n, const SweepArgs& a, int grid, hipStream_t stream) {
  if (a.nwork <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((sweep_kernel<S, N>), dim3(grid), dim3(Geo<N>::T), 0, stream, a);
    return hipGetLastError();
  });
}

hipError_t launch_init(int storage, int n, void* buf, const double* rho, const double* u, int64_t ncells,
                       hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((init_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream, static_cast<S*>(buf),
                       rho, u, ncells);
    return hipGetLastError();
  });
}

hipError_t launch_moments(int storage, int n, const void* buf, double* rho, double* u, int64_t ncells,
                          hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((moments_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream,
                       static_cast<const S*>(buf), rho, u, ncells);
    return hipGetLastError();
  });
}

hipError_t launch_get_pdfs(int storage, int n, const void* buf, double* h, int64_t ncells, hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((get_pdfs_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream,
                       static_cast<const S*>(buf), h, ncells);
    return hipGetLastError();
  });
}

hipError_t launch_set_pdfs(int storage, int n, void* buf, const double* h, int64_t ncells, hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((set_pdfs_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream,
                       static_cast<S*>(buf), h, ncells);
    return hipGetLastError();
  });
}

hipError_t launch_reduce(int storage, int n, const void* buf, int64_t ncells, double* out, hipStream_t stream) {
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((reduce_kernel<S, N>), dim3(kReduceGrid), dim3(kReduceThreads), 0, stream,
                       static_cast<const S*>(buf), ncells, out);
    return hipGetLastError();
  });
}

}  // namespace lbm
