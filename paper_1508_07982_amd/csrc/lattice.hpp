// Device-side lattice constants, storage forms and vector access shared by
// the HIP kernels of the library.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace lbm {
namespace dev {

// ---- D3Q19 velocity set (rest, 6 faces, 12 edges; opposites adjacent) ----
__host__ __device__ __forceinline__ constexpr int ex(int a) {
  return a == 1 || a == 7 || a == 9 || a == 11 || a == 13 ? 1 : (a == 2 || a == 8 || a == 10 || a == 12 || a == 14 ? -1 : 0);
}
__host__ __device__ __forceinline__ constexpr int ey(int a) {
  return a == 3 || a == 7 || a == 10 || a == 15 || a == 17 ? 1 : (a == 4 || a == 8 || a == 9 || a == 16 || a == 18 ? -1 : 0);
}
__host__ __device__ __forceinline__ constexpr int ez(int a) {
  return a == 5 || a == 11 || a == 14 || a == 15 || a == 18 ? 1 : (a == 6 || a == 12 || a == 13 || a == 16 || a == 17 ? -1 : 0);
}
// the opposite direction: pairs (a, a + 1) for odd a
__host__ __device__ __forceinline__ constexpr int opp(int a) { return a == 0 ? 0 : (a & 1 ? a + 1 : a - 1); }
constexpr bool opp_is_opposite() {
  for (int a = 0; a < 19; ++a)
    if (ex(opp(a)) != -ex(a) || ey(opp(a)) != -ey(a) || ez(opp(a)) != -ez(a)) return false;
  return true;
}
static_assert(opp_is_opposite(), "opposite directions");

template <typename C>
__host__ __device__ __forceinline__ constexpr C wgt(int a) {
  return a == 0 ? C(1) / C(3) : (a <= 6 ? C(1) / C(18) : C(1) / C(36));
}

// ---- PDF layout --------------------------------------------------------------
// A level buffer is block-major: block `slot` holds its 19 direction planes
// of n^3 cells one after the other, element (a, slot, cell) at
// (19 slot + a) n^3 + cell.  The 19 rows a tile reads then lie inside one
// block's 19 n^3 elements, which measured faster than direction planes
// spanning the whole level.  Interior cells keep their canonical index
// idx = slot * n^3 + cell.
constexpr int kQ = 19;
template <int N>
__host__ __device__ constexpr uint64_t pdf_index(int a, uint64_t slot, uint32_t cell) {
  return (slot * kQ + uint64_t(a)) * uint64_t(N * N * N) + cell;
}
template <int N>
__host__ __device__ constexpr uint64_t pdf_at(int a, uint64_t idx) {
  constexpr uint64_t N3 = uint64_t(N) * N * N;
  return (idx / N3 * kQ + uint64_t(a)) * N3 + idx % N3;
}
// the same for a block size known only at run time
__host__ __device__ inline uint64_t pdf_at_rt(int a, uint64_t idx, uint64_t n3) {
  return (idx / n3 * kQ + uint64_t(a)) * n3 + idx % n3;
}

// ---- x faces ----------------------------------------------------------------
// Values that cross a block's x faces (cells x = 0 or n - 1 of one direction)
// are n apart in the block-major layout, one element per 128-byte line.
// Where a kernel reads or writes many of them, they are kept in an x-face
// buffer instead: one element per (row, x direction, y, z), the 10
// directions with a nonzero x component numbered in direction order.  The
// (j, k) rows jk = j + n k come in groups of G rows, each group holding its
// rows for all 10 directions: element (row, q, jk) at 10 n^2 row +
// 10 G (jk / G) + G q + jk mod G.  FP64 and FP32 take G = 32 bytes /
// element size (4 and 8: the rows of a 64-lane workgroup of the sweep at
// n = 32), so that the face values one workgroup writes form one contiguous
// run of whole 64-byte segments; FP16 takes G = n^2 (one group per face,
// direction after direction), which measured faster for its packed sweep.
constexpr int kXDirs = 10;
__host__ __device__ __forceinline__ constexpr int xdir_index(int a) {
  int q = 0;
  for (int b = 0; b < a; ++b) q += ex(b) != 0 ? 1 : 0;
  return q;
}
// the direction with x-direction number q
__host__ __device__ __forceinline__ constexpr int xdir_dir(int q) {
  int a = 0;
  for (int seen = -1; a < 19; ++a) {
    seen += ex(a) != 0 ? 1 : 0;
    if (ex(a) != 0 && seen == q) break;
  }
  return a;
}
// rows per group of the x-face layout for element type S and block size n
template <typename S>
__host__ __device__ constexpr int face_rows(int n) {
  return sizeof(S) == 2 ? n * n : 32 / int(sizeof(S));
}
// element (row, q, jk): q the x-direction number
template <typename S, int N>
__host__ __device__ __forceinline__ uint64_t xface_at(uint64_t row, int q, uint32_t jk) {
  constexpr uint32_t G = uint32_t(face_rows<S>(N));
  static_assert((N * N) % G == 0, "a whole number of row groups per face");
  return row * uint64_t(kXDirs * N * N) + uint64_t(jk / G) * (kXDirs * G) + uint64_t(q) * G + (jk % G);
}
// the inverse, for a block size known only at run time: element e -> (row, q, jk)
template <typename S>
__host__ __device__ __forceinline__ void xface_decode(int64_t e, int n, int64_t& row, int& q, int64_t& jk) {
  const int64_t G = face_rows<S>(n);
  const int64_t per = int64_t(kXDirs) * n * n, r = e % per;
  row = e / per;
  q = int((r % (kXDirs * G)) / G);
  jk = (r / (kXDirs * G)) * G + r % G;
}
// element (row, xdir_index(A), jk), A known at compile time
template <typename S, int N, int A>
__device__ __forceinline__ uint64_t xface_index(uint64_t row, uint32_t jk) {
  return xface_at<S, N>(row, xdir_index(A), jk);
}
// the same for a direction known only at run time
__host__ __device__ __forceinline__ constexpr int xdir_index_rt(int a) {
  // directions 1, 2 and 7 .. 14 have a nonzero x component
  return a <= 2 ? a - 1 : a - 5;
}
template <typename S, int N>
__device__ __forceinline__ uint64_t xface_index_rt(int a, uint64_t row, uint32_t jk) {
  return xface_at<S, N>(row, xdir_index_rt(a), jk);
}
static_assert(xdir_index(1) == 0 && xdir_index(2) == 1 && xdir_index(7) == 2 && xdir_index(14) == 9, "x directions");
constexpr bool xdir_rt_matches() {
  for (int a = 0; a < 19; ++a)
    if (ex(a) != 0 && xdir_index_rt(a) != xdir_index(a)) return false;
  return true;
}
static_assert(xdir_rt_matches(), "x directions");
static_assert(xdir_dir(0) == 1 && xdir_dir(1) == 2 && xdir_dir(2) == 7 && xdir_dir(9) == 14, "x directions");

// ---- storage forms --------------------------------------------------------
// A value bound for FP16 storage is first rounded to FP32: without the empty
// asm the compiler may fuse a collision's last multiply-add and the
// conversion into one mixed-precision instruction (a single rounding) in one
// kernel and not in another, and kernels that must agree bitwise would not.
__device__ __forceinline__ float keep_fp32(float v) {
  asm("" : "+v"(v));
  return v;
}

template <typename S>
struct Form;
template <>
struct Form<double> {
  using C = double;
  static __device__ __forceinline__ double ld(const double* p) { return *p; }
  static __device__ __forceinline__ void st(double* p, double v) { *p = v; }
  static __device__ __forceinline__ double omega(const SweepArgs& a) { return a.omega64; }
  static __device__ __forceinline__ double lambda_o(const SweepArgs& a) { return a.lambda_o64; }
  static __device__ __forceinline__ double accel(const SweepArgs& a, int d) { return a.accel64[d]; }
};
template <>
struct Form<float> {
  using C = float;
  static __device__ __forceinline__ float ld(const float* p) { return *p; }
  static __device__ __forceinline__ void st(float* p, float v) { *p = v; }
  static __device__ __forceinline__ float omega(const SweepArgs& a) { return a.omega; }
  static __device__ __forceinline__ float lambda_o(const SweepArgs& a) { return a.lambda_o; }
  static __device__ __forceinline__ float accel(const SweepArgs& a, int d) { return a.accel[d]; }
};
template <>
struct Form<__half> {
  using C = float;
  static __device__ __forceinline__ float ld(const __half* p) { return __half2float(*p); }
  static __device__ __forceinline__ void st(__half* p, float v) { *p = __float2half_rn(keep_fp32(v)); }
  static __device__ __forceinline__ float omega(const SweepArgs& a) { return a.omega; }
  static __device__ __forceinline__ float lambda_o(const SweepArgs& a) { return a.lambda_o; }
  static __device__ __forceinline__ float accel(const SweepArgs& a, int d) { return a.accel[d]; }
};

// ---- vector access: W consecutive cells of one row per lane ----------------
// Stores are nontemporal: the sweep's output is not read again before the
// next launch, and streaming it past the caches measured faster.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename S>
struct Vec;
template <>
struct Vec<float> {
  static constexpr int W = 4;  // 16-byte loads and stores
  static __device__ __forceinline__ void load(const float* p, float* v) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x, v[1] = t.y, v[2] = t.z, v[3] = t.w;
  }
  static __device__ __forceinline__ void store(float* p, const float* v) {
    const f32x4 t = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(t, reinterpret_cast<f32x4*>(p));
  }
};
template <>
struct Vec<double> {
  static constexpr int W = 2;  // 16-byte loads and stores
  static __device__ __forceinline__ void load(const double* p, double* v) {
    const double2 t = *reinterpret_cast<const double2*>(p);
    v[0] = t.x, v[1] = t.y;
  }
  static __device__ __forceinline__ void store(double* p, const double* v) {
    const f64x2 t = {v[0], v[1]};
    __builtin_nontemporal_store(t, reinterpret_cast<f64x2*>(p));
  }
};
template <>
struct Vec<__half> {
  static constexpr int W = 4;  // 8-byte loads and stores
  static __device__ __forceinline__ void load(const __half* p, float* v) {
    const uint2 t = *reinterpret_cast<const uint2*>(p);
    v[0] = __half2float(__ushort_as_half(uint16_t(t.x & 0xFFFFu)));
    v[1] = __half2float(__ushort_as_half(uint16_t(t.x >> 16)));
    v[2] = __half2float(__ushort_as_half(uint16_t(t.y & 0xFFFFu)));
    v[3] = __half2float(__ushort_as_half(uint16_t(t.y >> 16)));
  }
  static __device__ __forceinline__ void store(__half* p, const float* v) {
    u32x2 t;
    t.x = uint32_t(__half_as_ushort(__float2half_rn(keep_fp32(v[0])))) |
          (uint32_t(__half_as_ushort(__float2half_rn(keep_fp32(v[1])))) << 16);
    t.y = uint32_t(__half_as_ushort(__float2half_rn(keep_fp32(v[2])))) |
          (uint32_t(__half_as_ushort(__float2half_rn(keep_fp32(v[3])))) << 16);
    __builtin_nontemporal_store(t, reinterpret_cast<u32x2*>(p));
  }
};

// Cross-lane moves inside 16-lane DPP rows: lane l receives lane l - 1
// (shift right) or lane l + 1 (shift left).  A cell row of N cells spans
// N / W <= 16 lanes, aligned to the DPP rows, and the lanes at the two ends
// of a cell row take their outside value from a separate load.
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShl1 = 0x101;
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xFFFFFFFFll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(uint32_t(lo)) | ((long long)hi << 32));
}

// Cells per lane: FP16 blocks of 8 or more cells per row keep 8 cells per
// lane as packed pairs (16-byte accesses, see the packed path of the sweep);
// otherwise the storage form's vector width.
template <typename S, int N>
struct Geo {
  static constexpr bool PACKED = sizeof(S) == 2 && N >= 8;
  static constexpr int W = PACKED ? 8 : Vec<S>::W;
  static constexpr int N3 = N * N * N;
  static constexpr int CELLS = N3 < 256 * W ? N3 : 256 * W;  // cells per work tile
  static constexpr int T = CELLS / W;                          // threads per workgroup
  static constexpr int TPB = N3 / CELLS;                       // tiles per block
  static constexpr int H = N / 2;
  static_assert(N / W <= 16, "a cell row must fit one DPP row");
};

// ---- interpolated explosion ------------------------------------------------
// The exploded value of a fine ghost cell in the interpolated form: each PDF
// is reconstructed linearly inside its coarse parent P (the interpolation of
// exploded values of Algorithm 2, section 4.1, read as a limited linear
// reconstruction): f_a(P) + sum_d (o_d - 1/2) / 2 g_d, o the cell's octant in
// P, g_d = minmod(f(P + e_d) - f(P), f(P) - f(P - e_d)), and g_d = 0 where a
// face neighbour of P is no interior cell of P's level.  The 8 children of a
// parent average to its value, and zero slopes give eq. ctof.
template <typename C>
__device__ __forceinline__ C minmod(C p, C q) {
  return p * q <= C(0) ? C(0) : (fabs(p) < fabs(q) ? p : q);
}

// The reconstruction from P's value f[0] and its face neighbours' f[1 + 2d]
// (P + e_d) and f[2 + 2d] (P - e_d); b[q] < 0 marks a neighbour that is no
// interior cell (no slope along that axis).
template <typename C>
__device__ __forceinline__ C interp_combine(const C* f, const int* b, int ox, int oy, int oz) {
  C v = f[0];
  const int o[3] = {ox, oy, oz};
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (b[1 + 2 * d] >= 0 && b[2 + 2 * d] >= 0)
      v += (C(o[d]) - C(0.5)) * C(0.5) * minmod<C>(f[1 + 2 * d] - f[0], f[0] - f[2 + 2 * d]);
  return v;
}
// Offset q of the 7 positions of a reconstruction: P, then P + e_d and
// P - e_d for d = x, y, z.
__device__ __forceinline__ int interp_dx(int q, int d) {
  const int axis = (q - 1) >> 1, s = q == 0 ? 0 : (q & 1 ? 1 : -1);
  return axis == d ? s : 0;
}

// P = (px, py, pz): local coordinates relative to the block whose 27-entry
// neighbour table is `tab` (entry 13: that block), at most one block away
// (coordinates in [-N, 2N), neighbours included); buf is P's level buffer.
// A P outside every block of that level sets an error bit and gives 0.  The
// 7 table entries are loaded together, then the 7 values (a position that is
// no block reads element 0 instead, and its value is not used), so that a
// reconstruction costs two memory round trips.
template <typename S, int N>
__device__ inline typename Form<S>::C interp_value(const S* buf, const int32_t* tab, int px, int py, int pz, int a,
                                                  int ox, int oy, int oz, int* err) {
  using C = typename Form<S>::C;
  auto sd = [](int c) { return c < 0 ? -1 : (c >= N ? 1 : 0); };
  int x[7], y[7], z[7], b[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    x[q] = px + interp_dx(q, 0);
    y[q] = py + interp_dx(q, 1);
    z[q] = pz + interp_dx(q, 2);
    b[q] = tab[13 + sd(x[q]) + 3 * sd(y[q]) + 9 * sd(z[q])];
  }
  C f[7];
#pragma unroll
  for (int q = 0; q < 7; ++q)
    f[q] = Form<S>::ld(buf + (b[q] >= 0 ? pdf_index<N>(a, uint32_t(b[q]), uint32_t((x[q] & (N - 1)) +
                                                                                 N * ((y[q] & (N - 1)) + N * (z[q] & (N - 1)))))
                                        : 0));
  if (b[0] < 0) {
    atomicOr(err, 1);
    return C(0);
  }
  return interp_combine<C>(f, b, ox, oy, oz);
}

}  // namespace dev
}  // namespace lbm
