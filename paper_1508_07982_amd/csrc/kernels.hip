// HIP helper kernels of the library (initial state, moments, raw PDF I/O,
// FP64 reductions) and the storage dispatch of the sweep.  PDF buffers are
// block-major: element (a, slot, cell) at (19 slot + a) n^3 + cell; interior
// cells of a level are addressed by their canonical index slot * n^3 + cell.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "coalesce.hpp"
#include "forest.hpp"
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

// Coalescence launch: one chunk per workgroup of kCoalChunk lanes, one pair
// per lane (coalesce_chunk in coalesce.hpp).  Walls and the interpolated
// explosion each have a variant of their own, so the periodic form with the
// homogeneous explosion carries no code for them.
template <typename S, int N, bool INTERP, bool WALLS>
__global__ void __launch_bounds__(kCoalChunk) coalesce_kernel(CoalArgs c) {
  __shared__ int32_t fns[8 * 27];
  __shared__ int32_t nbs[27];
  coalesce_chunk<S, N, INTERP, WALLS>(c, int(blockIdx.x), fns, nbs);
}

// x-face copy of a buffer (see CoalArgs): one thread per element of xf.
template <typename S, int N>
__global__ void face_copy_kernel(const S* buf, S* xf, int64_t count) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  int64_t slot, jk;
  int q;
  xface_decode<S>(e, N, slot, q, jk);
  const int A = xdir_dir(q);
  xf[e] = buf[pdf_index<N>(A, uint64_t(slot), uint32_t((ex(A) < 0 ? 0 : N - 1) + N * int(jk)))];
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
      hipLaunchKernelGGL((coalesce_kernel<S, N, true, true>), dim3(a.nchunks), dim3(kCoalChunk), 0, stream, a);
    else if (a.interp)
      hipLaunchKernelGGL((coalesce_kernel<S, N, true, false>), dim3(a.nchunks), dim3(kCoalChunk), 0, stream, a);
    else if (a.walls)
      hipLaunchKernelGGL((coalesce_kernel<S, N, false, true>), dim3(a.nchunks), dim3(kCoalChunk), 0, stream, a);
    else
      hipLaunchKernelGGL((coalesce_kernel<S, N, false, false>), dim3(a.nchunks), dim3(kCoalChunk), 0, stream, a);
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
