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
// Memory layout per level: [direction][slot][z][y][x], one slot per block,
// so a 64-lane wavefront reads 64 consecutive cells of one direction, and a
// direction plane is addressed by a uniform base plus a 32-bit cell offset.
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

// ---- vector access: W consecutive cells of one row per lane ----------------
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
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
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
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
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
    uint2 t;
    t.x = uint32_t(__half_as_ushort(__float2half_rn(v[0]))) | (uint32_t(__half_as_ushort(__float2half_rn(v[1]))) << 16);
    t.y = uint32_t(__half_as_ushort(__float2half_rn(v[2]))) | (uint32_t(__half_as_ushort(__float2half_rn(v[3]))) << 16);
    *reinterpret_cast<uint2*>(p) = t;
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

template <typename S, int N>
struct Geo {
  static constexpr int W = Vec<S>::W;
  static constexpr int N3 = N * N * N;
  static constexpr int CELLS = N3 < 256 * W ? N3 : 256 * W;  // cells per work tile
  static constexpr int T = CELLS / W;                          // threads per workgroup
  static constexpr int TPB = N3 / CELLS;                       // tiles per block
  static constexpr int H = N / 2;
  static_assert(N / W <= 16, "a cell row must fit one DPP row");
};

// Per-workgroup copy of the slot's neighbour table.
struct SlotCache {
  int32_t nbr[27];
};

// Neighbour offset (-1, 0, +1) of a local coordinate after a shift.
template <int N>
__device__ __forceinline__ int side(int c) {
  return c < 0 ? -1 : (c >= N ? 1 : 0);
}

// Value at level-L cell (lx, ly, lz) of the virtual block whose neighbour
// table entry is `code` (< kNbrFine, i.e. inside a level-(L-1) leaf): the
// parent's post-collision value (homogeneous explosion, eq. ctof).
template <typename S, int N, int A>
__device__ __forceinline__ typename Form<S>::C parent_value(const SweepArgs& a, int code, int lx, int ly, int lz) {
  constexpr int N3 = Geo<S, N>::N3, H = Geo<S, N>::H;
  const int pp = kNbrCoarse0 - code;
  const int oc = pp & 7;
  const int px = (oc & 1 ? H : 0) + (lx >> 1), py = (oc & 2 ? H : 0) + (ly >> 1), pz = (oc & 4 ? H : 0) + (lz >> 1);
  const S* p = static_cast<const S*>(a.par) + A * a.plane_par + uint32_t(pp >> 3) * N3;
  return Form<S>::ld(p + px + N * (py + N * pz));
}

// Value of a special source of cell (i, j, k) of slot `slot`, direction A.
//
// Coalescence (eq. ftoc, co == true): the mean over the 8 children c of the
// cell of the value the child holds after the finer level's two substeps,
// i.e. what the second fine stream pulled into c from c - e_A:
//   c - e_A in a level-(L+1) block  -> that cell's state after substep 1;
//   otherwise c - e_A is a halo cell, whose first-substep value came from
//   c - 2 e_A: the fine state at t if that is a level-(L+1) cell, else the
//   exploded coarse value, which is this cell's ordinary source `regular`.
//
// Coarse source (the cell x - e_A lies in a level-(L-1) leaf):
//   substep 1: the exploded parent value of x - e_A;
//   substep 2: x - e_A is a halo cell whose first-substep value was pulled
//   from x - 2 e_A: the level's own state at t there, or the exploded parent
//   value if x - 2 e_A is also in the coarse region.
template <typename S, int N, int A>
__device__ __forceinline__ typename Form<S>::C special_value(const SweepArgs& a, const SlotCache& sc, int slot, int i,
                                                             int j, int k, bool co, typename Form<S>::C regular) {
  using C = typename Form<S>::C;
  constexpr int N3 = Geo<S, N>::N3, H = Geo<S, N>::H;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  if (co) {
    const int oct = (i >= H ? 1 : 0) | (j >= H ? 2 : 0) | (k >= H ? 4 : 0);
    const int row = a.fine_index[slot];
    if (row < 0) {
      atomicOr(a.err, kErrNoChild);
      return C(0);
    }
    const int32_t* fn = a.fine_nbr + (row * 8 + oct) * 27;
    const S* f1 = static_cast<const S*>(a.fine1) + A * a.plane_fine;
    const S* f0 = static_cast<const S*>(a.fine0) + A * a.plane_fine;
    const int cx = 2 * (i & (H - 1)), cy = 2 * (j & (H - 1)), cz = 2 * (k & (H - 1));
    C s = C(0);
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
      for (int oy = 0; oy < 2; ++oy)
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) {
          const int yx = cx + ox - EX, yy = cy + oy - EY, yz = cz + oz - EZ;
          const int fy = fn[13 + side<N>(yx) + 3 * side<N>(yy) + 9 * side<N>(yz)];
          if (fy >= 0) {
            s += Form<S>::ld(f1 + uint32_t(fy) * N3 + (yx & (N - 1)) + N * ((yy & (N - 1)) + N * (yz & (N - 1))));
          } else {
            const int zx = yx - EX, zy = yy - EY, zz = yz - EZ;
            const int fz = fn[13 + side<N>(zx) + 3 * side<N>(zy) + 9 * side<N>(zz)];
            if (fz >= 0)
              s += Form<S>::ld(f0 + uint32_t(fz) * N3 + (zx & (N - 1)) + N * ((zy & (N - 1)) + N * (zz & (N - 1))));
            else
              s += regular;
          }
        }
    return s * C(0.125);
  }
  const int sx = i - EX, sy = j - EY, sz = k - EZ;
  const int code = sc.nbr[13 + side<N>(sx) + 3 * side<N>(sy) + 9 * side<N>(sz)];
  if (code > kNbrCoarse0) {  // not a coarse region: never expected here
    atomicOr(a.err, kErrNoSource);
    return C(0);
  }
  if (a.substep == 1) return parent_value<S, N, A>(a, code, sx & (N - 1), sy & (N - 1), sz & (N - 1));
  const int zx = sx - EX, zy = sy - EY, zz = sz - EZ;
  const int cz = sc.nbr[13 + side<N>(zx) + 3 * side<N>(zy) + 9 * side<N>(zz)];
  if (cz >= 0) {
    const S* p = static_cast<const S*>(a.prev) + A * a.plane + uint32_t(cz) * N3;
    return Form<S>::ld(p + (zx & (N - 1)) + N * ((zy & (N - 1)) + N * (zz & (N - 1))));
  }
  if (cz > kNbrCoarse0) {
    atomicOr(a.err, kErrNoSource);
    return C(0);
  }
  return parent_value<S, N, A>(a, cz, zx & (N - 1), zy & (N - 1), zz & (N - 1));
}

// Ordinary pull of direction A for the W cells (i0 .. i0+W-1, j, k) of one
// lane: one vector load of the source row and, for x-shifted directions, a
// DPP move plus one edge load at the ends of the row.  A source block that is
// not a level-L block sets `odd` (the address is then replaced by the
// lane's own, so every load stays inside the buffer).
template <typename S, int N, int A, bool SIMPLE>
__device__ __forceinline__ void pull_dir(const SweepArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                         typename Form<S>::C (*h)[Geo<S, N>::W], uint32_t& odd) {
  using C = typename Form<S>::C;
  constexpr int W = Geo<S, N>::W, N3 = Geo<S, N>::N3;
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const int sy = j - EY, sz = k - EZ;
  const int oy = EY == 0 ? 0 : side<N>(sy);
  const int oz = EZ == 0 ? 0 : side<N>(sz);
  const uint32_t row = uint32_t(N * ((sy & (N - 1)) + N * (sz & (N - 1))));
  const int dmain = 13 + 3 * oy + 9 * oz;
  const int nbm = sc.nbr[dmain];
  if (!SIMPLE) odd |= uint32_t(nbm < 0);
  const S* __restrict__ base = static_cast<const S*>(a.cur) + A * a.plane;
  const uint32_t bm = uint32_t(SIMPLE || nbm >= 0 ? nbm : slot) * N3 + row;
  C v[W];
  Vec<S>::load(base + bm + i0, v);
  if (EX == 0) {
#pragma unroll
    for (int c = 0; c < W; ++c) h[A][c] = v[c];
  } else if (EX == 1) {  // source x - 1
    const C prev = dpp_move<kDppRowShr1>(v[W - 1]);
#pragma unroll
    for (int c = W - 1; c > 0; --c) h[A][c] = v[c - 1];
    h[A][0] = prev;
    if (i0 == 0) {
      const int nbx = sc.nbr[dmain - 1];
      if (!SIMPLE) odd |= uint32_t(nbx < 0);
      h[A][0] = Form<S>::ld(base + uint32_t(SIMPLE || nbx >= 0 ? nbx : slot) * N3 + row + (N - 1));
    }
  } else {  // source x + 1
    const C next = dpp_move<kDppRowShl1>(v[0]);
#pragma unroll
    for (int c = 0; c < W - 1; ++c) h[A][c] = v[c + 1];
    h[A][W - 1] = next;
    if (i0 == N - W) {
      const int nbx = sc.nbr[dmain + 1];
      if (!SIMPLE) odd |= uint32_t(nbx < 0);
      h[A][W - 1] = Form<S>::ld(base + uint32_t(SIMPLE || nbx >= 0 ? nbx : slot) * N3 + row);
    }
  }
}

template <typename S, int N, bool SIMPLE, int A = 0>
__device__ __forceinline__ void pull_all(const SweepArgs& a, const SlotCache& sc, int slot, int i0, int j, int k,
                                         typename Form<S>::C (*h)[Geo<S, N>::W], uint32_t& odd) {
  pull_dir<S, N, A, SIMPLE>(a, sc, slot, i0, j, k, h, odd);
  if constexpr (A + 1 < 19) pull_all<S, N, SIMPLE, A + 1>(a, sc, slot, i0, j, k, h, odd);
}

// Cells of a lane whose direction-A source is not an ordinary level-L read:
// bit c of the returned mask; bit c of `co` marks a coalesced pair, i.e.
// x - e_A or (edge directions) one of its axis projections in region(L+1).
template <int N, int W, int A>
__device__ __forceinline__ uint32_t special_cells(const SlotCache& sc, uint32_t fl, int i0, int j, int k,
                                                  uint32_t& co) {
  constexpr int EX = ex(A), EY = ey(A), EZ = ez(A);
  const int oy = EY == 0 ? 0 : side<N>(j - EY);
  const int oz = EZ == 0 ? 0 : side<N>(k - EZ);
  uint32_t spec = 0;
  co = 0;
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int ox = EX == 0 ? 0 : side<N>(i0 + c - EX);
    const int nb = sc.nbr[13 + ox + 3 * oy + 9 * oz];
    bool coal = false;
    if (fl & kHasFine) {
      coal = nb == kNbrFine;
      if (A >= 7) {
        const int dA = EX != 0 ? 13 + ox : 13 + 3 * oy;
        const int dB = EZ != 0 ? 13 + 9 * oz : 13 + 3 * oy;
        coal = coal || sc.nbr[dA] == kNbrFine || sc.nbr[dB] == kNbrFine;
      }
    }
    spec |= uint32_t(coal || nb < 0) << c;
    co |= uint32_t(coal) << c;
  }
  return spec;
}

template <typename S, int N, int A = 0>
__device__ __forceinline__ void fixups(const SweepArgs& a, const SlotCache& sc, int slot, uint32_t fl, int i0, int j,
                                       int k, typename Form<S>::C (*h)[Geo<S, N>::W]) {
  constexpr int W = Geo<S, N>::W;
  uint32_t co;
  const uint32_t spec = special_cells<N, W, A>(sc, fl, i0, j, k, co);
  if (spec) {
#pragma unroll
    for (int c = 0; c < W; ++c)
      if ((spec >> c) & 1u) h[A][c] = special_value<S, N, A>(a, sc, slot, i0 + c, j, k, (co >> c) & 1u, h[A][c]);
  }
  if constexpr (A + 1 < 19) fixups<S, N, A + 1>(a, sc, slot, fl, i0, j, k, h);
}

template <typename C, int W, int A = 0>
__device__ __forceinline__ void relax(C (*h)[W], int c, C drho, C ux, C uy, C uz, C usq, C om) {
  constexpr C w = wgt<C>(A);
  const C eu = C(ex(A)) * ux + C(ey(A)) * uy + C(ez(A)) * uz;
  const C heq = w * (drho + C(3) * eu + C(4.5) * eu * eu - usq);
  h[A][c] = h[A][c] + om * (heq - h[A][c]);
  if constexpr (A + 1 < 19) relax<C, W, A + 1>(h, c, drho, ux, uy, uz, usq, om);
}

// SRT collision of cell c in shifted form (rho0 = 1).
template <typename C, int W>
__device__ __forceinline__ void collide(C (*h)[W], int c, C om) {
  C drho = C(0), ux = C(0), uy = C(0), uz = C(0);
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    drho += h[a][c];
    if (ex(a)) ux += ex(a) > 0 ? h[a][c] : -h[a][c];
    if (ey(a)) uy += ey(a) > 0 ? h[a][c] : -h[a][c];
    if (ez(a)) uz += ez(a) > 0 ? h[a][c] : -h[a][c];
  }
  const C usq = C(1.5) * (ux * ux + uy * uy + uz * uz);
  relax<C, W>(h, c, drho, ux, uy, uz, usq, om);
}

template <typename S, int N, bool SIMPLE>
__device__ __forceinline__ void update_lane(const SweepArgs& a, const SlotCache& sc, int slot, uint32_t fl, int cell0) {
  using C = typename Form<S>::C;
  constexpr int W = Geo<S, N>::W, N3 = Geo<S, N>::N3;
  const int i0 = cell0 & (N - 1), j = (cell0 / N) & (N - 1), k = cell0 / (N * N);
  C h[19][W];
  uint32_t odd = 0;
  pull_all<S, N, SIMPLE>(a, sc, slot, i0, j, k, h, odd);
  if (!SIMPLE && odd) fixups<S, N>(a, sc, slot, fl, i0, j, k, h);
  const C om = Form<S>::omega(a);
#pragma unroll
  for (int c = 0; c < W; ++c) collide<C, W>(h, c, om);
  S* __restrict__ nxt = static_cast<S*>(a.nxt) + uint32_t(slot) * N3 + uint32_t(cell0);
#pragma unroll
  for (int d = 0; d < 19; ++d) Vec<S>::store(nxt + d * a.plane, h[d]);
}

template <typename S, int N>
__device__ __forceinline__ void sweep_item(const SweepArgs& a, SlotCache& sc, int w) {
  constexpr int W = Geo<S, N>::W, CELLS = Geo<S, N>::CELLS, TPB = Geo<S, N>::TPB;
  const int item = a.work[w];
  const int slot = item / TPB;
  const int cell0 = (item - slot * TPB) * CELLS + int(threadIdx.x) * W;
  if (threadIdx.x < 27) sc.nbr[threadIdx.x] = a.nbr[slot * 27 + threadIdx.x];
  __syncthreads();
  const uint32_t fl = a.flags[slot];
  if (fl & kAllSameLevel)
    update_lane<S, N, true>(a, sc, slot, fl, cell0);
  else
    update_lane<S, N, false>(a, sc, slot, fl, cell0);
}

// One workgroup per work tile (PERSIST = false), or a fixed grid of
// workgroups looping over the tiles (PERSIST = true).
template <typename S, int N, bool PERSIST>
__global__ void __launch_bounds__((Geo<S, N>::T)) sweep_kernel(SweepArgs a) {
  __shared__ SlotCache sc;
  if (!PERSIST) {
    sweep_item<S, N>(a, sc, blockIdx.x);
    return;
  }
  for (int w = blockIdx.x; w < a.nwork; w += gridDim.x) {
    sweep_item<S, N>(a, sc, w);
    __syncthreads();
  }
}

// ---- init / moments / raw I/O / reductions -------------------------------

template <typename S, int N>
__global__ void init_kernel(S* buf, uint64_t plane, const double* rho, const double* u, int64_t ncells) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
  const double r = rho[idx], ux = u[3 * idx], uy = u[3 * idx + 1], uz = u[3 * idx + 2];
  const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    const double eu = ex(a) * ux + ey(a) * uy + ez(a) * uz;
    const double h = wgt<double>(a) * ((r - 1.0) + 3.0 * eu + 4.5 * eu * eu - usq);
    Form<S>::st(buf + a * plane + idx, typename Form<S>::C(h));
  }
}

template <typename S, int N>
__global__ void moments_kernel(const S* buf, uint64_t plane, double* rho, double* u, int64_t ncells) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
  double s = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    const double h = double(Form<S>::ld(buf + a * plane + idx));
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
__global__ void get_pdfs_kernel(const S* buf, uint64_t plane, double* h, int64_t ncells) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
#pragma unroll
  for (int a = 0; a < 19; ++a) h[idx * 19 + a] = double(Form<S>::ld(buf + a * plane + idx));
}

template <typename S, int N>
__global__ void set_pdfs_kernel(S* buf, uint64_t plane, const double* h, int64_t ncells) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncells) return;
#pragma unroll
  for (int a = 0; a < 19; ++a)
    Form<S>::st(buf + a * plane + idx, typename Form<S>::C(h[idx * 19 + a]));
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
__global__ void __launch_bounds__(kReduceThreads) reduce_kernel(const S* buf, uint64_t plane, int64_t ncells,
                                                                double* out) {
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < ncells;
       idx += int64_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      const double h = double(Form<S>::ld(buf + a * plane + idx));
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

int sweep_tile_cells(int storage, int n) {
  const int n3 = n * n * n;
  const int w = storage == 0 ? Vec<double>::W : Vec<float>::W;
  return n3 < 256 * w ? n3 : 256 * w;
}

hipError_t launch_sweep(int storage, int n, const SweepArgs& a, int grid, hipStream_t stream) {
  if (a.nwork <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    if (grid >= a.nwork)
      hipLaunchKernelGGL((sweep_kernel<S, N, false>), dim3(a.nwork), dim3(Geo<S, N>::T), 0, stream, a);
    else
      hipLaunchKernelGGL((sweep_kernel<S, N, true>), dim3(grid), dim3(Geo<S, N>::T), 0, stream, a);
    return hipGetLastError();
  });
}

hipError_t launch_init(int storage, int n, void* buf, uint64_t plane, const double* rho, const double* u,
                       int64_t ncells, hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((init_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream, static_cast<S*>(buf),
                       plane, rho, u, ncells);
    return hipGetLastError();
  });
}

hipError_t launch_moments(int storage, int n, const void* buf, uint64_t plane, double* rho, double* u,
                          int64_t ncells, hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((moments_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream,
                       static_cast<const S*>(buf), plane, rho, u, ncells);
    return hipGetLastError();
  });
}

hipError_t launch_get_pdfs(int storage, int n, const void* buf, uint64_t plane, double* h, int64_t ncells,
                           hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((get_pdfs_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream,
                       static_cast<const S*>(buf), plane, h, ncells);
    return hipGetLastError();
  });
}

hipError_t launch_set_pdfs(int storage, int n, void* buf, uint64_t plane, const double* h, int64_t ncells,
                           hipStream_t stream) {
  if (ncells <= 0) return hipSuccess;
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((set_pdfs_kernel<S, N>), dim3(grid_for(ncells, 256)), dim3(256), 0, stream,
                       static_cast<S*>(buf), plane, h, ncells);
    return hipGetLastError();
  });
}

hipError_t launch_reduce(int storage, int n, const void* buf, uint64_t plane, int64_t ncells, double* out,
                         hipStream_t stream) {
  return dispatch(storage, n, [&](auto s, auto nn) {
    using S = decltype(s);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((reduce_kernel<S, N>), dim3(kReduceGrid), dim3(kReduceThreads), 0, stream,
                       static_cast<const S*>(buf), plane, ncells, out);
    return hipGetLastError();
  });
}

}  // namespace lbm
