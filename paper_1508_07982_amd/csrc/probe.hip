// Bandwidth probes (declared in lbm_probe.h): a 16-byte copy and the sweep's
// access shape without arithmetic, timed with HIP events on the caller's
// stream.  They allocate nothing.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbm_probe.h"
#include "../../include/lbm_refined.h"

namespace lbm {
int set_error(int code, const char* fmt, ...);
}

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void __launch_bounds__(256) copy_kernel(u32x4* __restrict__ dst, const u32x4* __restrict__ src,
                                                   int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x) {
    const u32x4 v = src[i];
    if (NT)
      __builtin_nontemporal_store(v, dst + i);
    else
      dst[i] = v;
  }
}

// Workgroup b -> tile such that each of the 8 XCDs (workgroups dispatched
// round-robin) takes one contiguous range of tiles; a bijection of [0, n).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n) {
  const int64_t x = b & 7, r = b >> 3, q = n >> 3, rem = n & 7;
  return x * q + (x < rem ? x : rem) + r;
}

// One workgroup per tile of LANES * (16 / elem bytes) cells of one block:
// 19 row loads of 16 bytes per lane, then 19 nontemporal stores.
template <int LANES>
__global__ void __launch_bounds__(LANES) streams_kernel(u32x4* __restrict__ dst, const u32x4* __restrict__ src,
                                                        int64_t tiles, int64_t tiles_per_block, int64_t row16,
                                                        int xcd) {
  const int64_t t = xcd ? xcd_tile(blockIdx.x, tiles) : int64_t(blockIdx.x);
  const int64_t blk = t / tiles_per_block;
  const int64_t off = (t - blk * tiles_per_block) * LANES + threadIdx.x;  // 16-byte unit inside a row
  const int64_t base = blk * 19 * row16 + off;
  u32x4 v[19];
#pragma unroll
  for (int a = 0; a < 19; ++a) v[a] = src[base + a * row16];
#pragma unroll
  for (int a = 0; a < 19; ++a) __builtin_nontemporal_store(v[a], dst + base + a * row16);
}

struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

int hip_fail(hipError_t e, const char* what) { return lbm::set_error(LBM_E_HIP, "%s: %s", what, hipGetErrorString(e)); }

}  // namespace

extern "C" {

int lbm_probe_copy(void* dst, const void* src, int64_t bytes, int iters, int nontemporal, void* stream, double* ms) {
  if (!dst || !src || !ms) return lbm::set_error(LBM_E_INVALID, "null pointer");
  if (bytes <= 0 || bytes % 16 || iters < 1) return lbm::set_error(LBM_E_INVALID, "bytes must be a positive multiple of 16, iters >= 1");
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return lbm::set_error(LBM_E_INVALID, "buffers must be 16-byte aligned");
  const uintptr_t d0 = reinterpret_cast<uintptr_t>(dst), s0 = reinterpret_cast<uintptr_t>(src);
  if (d0 < s0 + uint64_t(bytes) && s0 < d0 + uint64_t(bytes)) return lbm::set_error(LBM_E_INVALID, "buffers overlap");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t count = bytes / 16;
  const int64_t want = (count + 255) / 256;
  const unsigned grid = unsigned(want < 65536 * 4 ? want : 65536 * 4);
  Events ev;
  hipError_t e;
  if ((e = hipEventCreate(&ev.e0)) || (e = hipEventCreate(&ev.e1))) return hip_fail(e, "hipEventCreate");
  auto launch = [&]() {
    if (nontemporal)
      hipLaunchKernelGGL(copy_kernel<true>, dim3(grid), dim3(256), 0, s, static_cast<u32x4*>(dst),
                         static_cast<const u32x4*>(src), count);
    else
      hipLaunchKernelGGL(copy_kernel<false>, dim3(grid), dim3(256), 0, s, static_cast<u32x4*>(dst),
                         static_cast<const u32x4*>(src), count);
    return hipGetLastError();
  };
  if ((e = launch())) return hip_fail(e, "copy launch");  // warm-up
  if ((e = hipEventRecord(ev.e0, s))) return hip_fail(e, "hipEventRecord");
  for (int i = 0; i < iters; ++i)
    if ((e = launch())) return hip_fail(e, "copy launch");
  if ((e = hipEventRecord(ev.e1, s))) return hip_fail(e, "hipEventRecord");
  if ((e = hipStreamSynchronize(s))) return hip_fail(e, "hipStreamSynchronize");
  float t = 0.f;
  if ((e = hipEventElapsedTime(&t, ev.e0, ev.e1))) return hip_fail(e, "hipEventElapsedTime");
  *ms = double(t) / iters;
  return LBM_OK;
}

int lbm_probe_streams(void* dst, const void* src, int64_t nblocks, int cells_per_block, int elem_bytes, int lanes,
                      int xcd, int iters, void* stream, double* ms) {
  if (!dst || !src || !ms) return lbm::set_error(LBM_E_INVALID, "null pointer");
  const int n = cells_per_block;
  if ((n != 16 && n != 32) || (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) ||
      (lanes != 64 && lanes != 128 && lanes != 256) || nblocks < 1 || iters < 1)
    return lbm::set_error(LBM_E_INVALID, "bad probe parameters");
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return lbm::set_error(LBM_E_INVALID, "buffers must be 16-byte aligned");
  const int64_t row16 = int64_t(n) * n * n * elem_bytes / 16;  // 16-byte units per direction row of a block
  if (row16 % lanes) return lbm::set_error(LBM_E_INVALID, "a block row must hold whole tiles");
  const int64_t tiles_per_block = row16 / lanes;
  const int64_t tiles = nblocks * tiles_per_block;
  if (tiles > 0x7fffffff) return lbm::set_error(LBM_E_INVALID, "too many tiles");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Events ev;
  hipError_t e;
  if ((e = hipEventCreate(&ev.e0)) || (e = hipEventCreate(&ev.e1))) return hip_fail(e, "hipEventCreate");
  auto launch = [&]() {
    u32x4* d = static_cast<u32x4*>(dst);
    const u32x4* q = static_cast<const u32x4*>(src);
    if (lanes == 64)
      hipLaunchKernelGGL(streams_kernel<64>, dim3(unsigned(tiles)), dim3(64), 0, s, d, q, tiles, tiles_per_block, row16, xcd);
    else if (lanes == 128)
      hipLaunchKernelGGL(streams_kernel<128>, dim3(unsigned(tiles)), dim3(128), 0, s, d, q, tiles, tiles_per_block, row16, xcd);
    else
      hipLaunchKernelGGL(streams_kernel<256>, dim3(unsigned(tiles)), dim3(256), 0, s, d, q, tiles, tiles_per_block, row16, xcd);
    return hipGetLastError();
  };
  if ((e = launch())) return hip_fail(e, "probe launch");  // warm-up
  if ((e = hipEventRecord(ev.e0, s))) return hip_fail(e, "hipEventRecord");
  for (int i = 0; i < iters; ++i)
    if ((e = launch())) return hip_fail(e, "probe launch");
  if ((e = hipEventRecord(ev.e1, s))) return hip_fail(e, "hipEventRecord");
  if ((e = hipStreamSynchronize(s))) return hip_fail(e, "hipStreamSynchronize");
  float t = 0.f;
  if ((e = hipEventElapsedTime(&t, ev.e0, ev.e1))) return hip_fail(e, "hipEventElapsedTime");
  *ms = double(t) / iters;
  return LBM_OK;
}

}  // extern "C"
