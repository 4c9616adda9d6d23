// Refinement indicators and the learned surrogate (C ABI in lbm_refined.h).
//
// The paper refines statically and leaves the criterion to the user's
// callbacks (section 3.3); dynamic refinement is named future work
// (section 6).  Definitions used here, per block, on the stored
// (post-collision) state:
//
//   per cell  rho, u (eq. fvelocity), f_eq (eq. fequ), neq = ||f - f_eq|| / rho,
//             |curl u| with block-local differences in the block's lattice
//             units (central inside, one-sided on the block faces);
//   criterion I_omega = max |curl u|, I_neq = mean neq; refine-worthy if
//             I_omega > theta_omega or I_neq > theta_neq, coarsen-worthy if both
//             are below half their threshold, keep otherwise;
//   features  (12) level / Lmax, 1e3 mean(rho - 1), and log10(x + 1e-12) of
//             std rho, |mean u|, rms |u - mean u|, max |u|, the octant-mean
//             jumps of u along x, y, z, |curl| of the 2x2x2 octant-mean field,
//             mean neq, max neq.
//
// The surrogate is an MLP 12 -> 64 -> 64 -> 1 (ReLU, sigmoid) in FP32 with
// hand-written forward, backward and Adam kernels; its output p is a soft
// version of the criterion's target (1 refine, 0.5 keep, 0 coarsen).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/lbm_refined.h"
#include "lattice.hpp"
#include "state.hpp"

using namespace lbm;
using namespace lbm::dev;

namespace {

constexpr int kFeat = 12;
constexpr int kHid = 64;
constexpr int kParams = kHid * kFeat + kHid + kHid * kHid + kHid + kHid + 1;  // 5057
constexpr int oW1 = 0, oB1 = oW1 + kHid * kFeat, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid;

#define TRY(expr)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return set_error(e_ == hipErrorOutOfMemory ? LBM_E_OOM : LBM_E_HIP, \
                                           "%s: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

// ---- per-cell moments and non-equilibrium norm -----------------------------

// Cells of the listed blocks (all blocks when `blocks` is null); outputs
// are indexed like the level buffer (slot * n^3 + cell).
template <typename S>
__global__ void cell_stats_kernel(const S* buf, const int32_t* blocks, int64_t ncells, int n3,
                                  double* drho, double* u, double* neq) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ncells) return;
  const int64_t idx = blocks ? int64_t(blocks[t / n3]) * n3 + t % n3 : t;
  double h[19];
  double s = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    h[a] = double(Form<S>::ld(buf + pdf_at_rt(a, uint64_t(idx), uint64_t(n3))));
    s += h[a];
    jx += ex(a) * h[a];
    jy += ey(a) * h[a];
    jz += ez(a) * h[a];
  }
  const double usq = 1.5 * (jx * jx + jy * jy + jz * jz);
  double q = 0;
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    const double eu = ex(a) * jx + ey(a) * jy + ez(a) * jz;
    const double heq = wgt<double>(a) * (s + 3.0 * eu + 4.5 * eu * eu - usq);
    q += (h[a] - heq) * (h[a] - heq);
  }
  drho[idx] = s;
  u[3 * idx] = jx;
  u[3 * idx + 1] = jy;
  u[3 * idx + 2] = jz;
  neq[idx] = sqrt(q) / (1.0 + s);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

constexpr int kStatThreads = 256;
constexpr int kAcc = 34;  // accumulators per thread (see block_stats_kernel)

// Workgroup reduction of the accumulators and, in thread 0, the features
// and criterion values of the block (either output may be null).
__device__ void block_finish(double* acc, int n, double level_frac, double* fo, double* co_out) {
  __shared__ double part[kStatThreads / 64][kAcc];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q = 0; q < kAcc; ++q) {
    const bool is_max = q == 6 || q == 7 || q == 9;
    const double v = is_max ? wmax(acc[q]) : wsum(acc[q]);
    if (lane == 0) part[wv][q] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int n3 = n * n * n, h = n / 2;
  double t[kAcc];
  for (int q = 0; q < kAcc; ++q) {
    const bool is_max = q == 6 || q == 7 || q == 9;
    t[q] = part[0][q];
    for (int w = 1; w < kStatThreads / 64; ++w) t[q] = is_max ? fmax(t[q], part[w][q]) : t[q] + part[w][q];
  }
  const double inv = 1.0 / n3;
  const double mdr = t[0] * inv;
  const double stdr = sqrt(fmax(t[1] * inv - mdr * mdr, 0.0));
  const double ub[3] = {t[2] * inv, t[3] * inv, t[4] * inv};
  const double ubn = sqrt(ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
  const double rms = sqrt(fmax(t[5] * inv - ubn * ubn, 0.0));
  double om[8][3];
  for (int o = 0; o < 8; ++o)
    for (int c = 0; c < 3; ++c) om[o][c] = t[10 + 3 * o + c] * (8.0 * inv);
  double jump[3], grad[3][3];
  for (int ax = 0; ax < 3; ++ax) {
    double hi[3] = {0, 0, 0}, lo[3] = {0, 0, 0};
    for (int o = 0; o < 8; ++o)
      for (int c = 0; c < 3; ++c) ((o >> ax) & 1 ? hi : lo)[c] += 0.25 * om[o][c];
    double s2 = 0;
    for (int c = 0; c < 3; ++c) {
      s2 += (hi[c] - lo[c]) * (hi[c] - lo[c]);
      grad[ax][c] = (hi[c] - lo[c]) / h;
    }
    jump[ax] = sqrt(s2);
  }
  const double co[3] = {grad[1][2] - grad[2][1], grad[2][0] - grad[0][2], grad[0][1] - grad[1][0]};
  const double con = sqrt(co[0] * co[0] + co[1] * co[1] + co[2] * co[2]);
  const double raw[10] = {stdr, ubn, rms, t[6], jump[0], jump[1], jump[2], con, t[8] * inv, t[9]};
  if (fo) {
    fo[0] = level_frac;
    fo[1] = 1e3 * mdr;
    for (int q = 0; q < 10; ++q) fo[2 + q] = log10(raw[q] + 1e-12);
  }
  if (co_out) {
    co_out[0] = t[7];
    co_out[1] = t[8] * inv;
  }
}

// Features only, in one pass over the PDFs: no per-cell buffers and no
// stencil (the |curl| accumulator stays zero and is not used).
template <typename S>
__global__ void __launch_bounds__(kStatThreads) block_features_kernel(const S* buf, int n,
                                                                      int nblocks, double level_frac,
                                                                      int64_t first, double* feat) {
  const int b = blockIdx.x;
  if (b >= nblocks) return;
  const int n3 = n * n * n, h = n / 2;
  double acc[kAcc];
  for (int q = 0; q < kAcc; ++q) acc[q] = 0.0;
  for (int c = threadIdx.x; c < n3; c += kStatThreads) {
    const int64_t idx = int64_t(b) * n3 + c;
    double hv[19];
    double s = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      hv[a] = double(Form<S>::ld(buf + pdf_at_rt(a, uint64_t(idx), uint64_t(n3))));
      s += hv[a];
      jx += ex(a) * hv[a];
      jy += ey(a) * hv[a];
      jz += ez(a) * hv[a];
    }
    const double usq = 1.5 * (jx * jx + jy * jy + jz * jz);
    double q2 = 0;
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      const double eu = ex(a) * jx + ey(a) * jy + ez(a) * jz;
      const double heq = wgt<double>(a) * (s + 3.0 * eu + 4.5 * eu * eu - usq);
      q2 += (hv[a] - heq) * (hv[a] - heq);
    }
    const double q = sqrt(q2) / (1.0 + s);
    acc[0] += s;
    acc[1] += s * s;
    acc[2] += jx;
    acc[3] += jy;
    acc[4] += jz;
    const double u2 = jx * jx + jy * jy + jz * jz;
    acc[5] += u2;
    acc[6] = fmax(acc[6], sqrt(u2));
    acc[8] += q;
    acc[9] = fmax(acc[9], q);
    const int i = c % n, j = (c / n) % n, k = c / (n * n);
    const int oct = (i >= h ? 1 : 0) | (j >= h ? 2 : 0) | (k >= h ? 4 : 0);
    acc[10 + 3 * oct] += jx;
    acc[11 + 3 * oct] += jy;
    acc[12 + 3 * oct] += jz;
  }
  block_finish(acc, n, level_frac, feat + (first + b) * kFeat, nullptr);
}

// Blocks whose decision goes to the criterion: p within delta of a decision
// boundary, or a feature outside the training range.
__global__ void fallback_kernel(const double* feat, const float* prob, const double* fmin, const double* fmax_,
                                int nb, double delta, int8_t* fb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double p = prob[b];
  bool f = fabs(p - 0.75) < delta || fabs(p - 0.25) < delta;
  for (int q = 0; q < kFeat && !f; ++q) {
    const double x = feat[b * kFeat + q];
    f = x < fmin[q] || x > fmax_[q];
  }
  fb[b] = f ? 1 : 0;
}

// One workgroup per block: reductions over its cells, then features and
// criterion values.  The level's blocks start at `first` in the outputs.
__global__ void __launch_bounds__(kStatThreads) block_stats_kernel(const double* drho, const double* u,
                                                                   const double* neq, int n, const int32_t* blocks,
                                                                   int nblocks, double level_frac, int64_t first,
                                                                   double* feat, double* crit) {
  if (int(blockIdx.x) >= nblocks) return;
  const int b = blocks ? blocks[blockIdx.x] : int(blockIdx.x);
  const int n3 = n * n * n, h = n / 2;
  const int64_t base = int64_t(b) * n3;
  // acc: 0 sum drho, 1 sum drho^2, 2..4 sum u, 5 sum |u|^2, 6 max |u|, 7 max curl,
  //      8 sum neq, 9 max neq, 10..33 octant sums of u (8 x 3)
  double acc[kAcc];
  for (int q = 0; q < kAcc; ++q) acc[q] = 0.0;
  auto U = [&](int i, int j, int k, int c) { return u[3 * (base + i + n * (j + n * k)) + c]; };
  for (int c = threadIdx.x; c < n3; c += kStatThreads) {
    const int i = c % n, j = (c / n) % n, k = c / (n * n);
    const double r = drho[base + c];
    const double ux = U(i, j, k, 0), uy = U(i, j, k, 1), uz = U(i, j, k, 2);
    acc[0] += r;
    acc[1] += r * r;
    acc[2] += ux;
    acc[3] += uy;
    acc[4] += uz;
    const double u2 = ux * ux + uy * uy + uz * uz;
    acc[5] += u2;
    acc[6] = fmax(acc[6], sqrt(u2));
    // block-local derivative along one axis
    auto d = [&](int comp, int axis) {
      int lo[3] = {i, j, k}, hi[3] = {i, j, k};
      const int p = axis == 0 ? i : (axis == 1 ? j : k);
      double scale = 0.5;
      if (p == 0) {
        hi[axis] = 1;
        lo[axis] = 0;
        scale = 1.0;
      } else if (p == n - 1) {
        hi[axis] = n - 1;
        lo[axis] = n - 2;
        scale = 1.0;
      } else {
        hi[axis] = p + 1;
        lo[axis] = p - 1;
      }
      return scale * (U(hi[0], hi[1], hi[2], comp) - U(lo[0], lo[1], lo[2], comp));
    };
    const double cx = d(2, 1) - d(1, 2), cy = d(0, 2) - d(2, 0), cz = d(1, 0) - d(0, 1);
    acc[7] = fmax(acc[7], sqrt(cx * cx + cy * cy + cz * cz));
    const double q = neq[base + c];
    acc[8] += q;
    acc[9] = fmax(acc[9], q);
    const int oct = (i >= h ? 1 : 0) | (j >= h ? 2 : 0) | (k >= h ? 4 : 0);
    acc[10 + 3 * oct] += ux;
    acc[11 + 3 * oct] += uy;
    acc[12 + 3 * oct] += uz;
  }
  block_finish(acc, n, level_frac, feat ? feat + (first + b) * kFeat : nullptr,
               crit ? crit + 2 * (first + b) : nullptr);
}

// ---- decision -----------------------------------------------------------------

// flags: +1 split, -1 merge candidate, 0 keep.  With a probability array the
// surrogate decides (p > 0.75 refine, p < 0.25 coarsen) except for blocks
// marked in fb, which the criterion decides.
__global__ void decide_kernel(const double* crit, const float* prob, const int8_t* fb, const int32_t* level, int nb,
                              int max_level, double th_w, double th_n, int8_t* flags) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  int d;
  if (!prob || fb[b]) {
    const double Iw = crit[2 * b], In = crit[2 * b + 1];
    d = 0;
    if (Iw > th_w || In > th_n)
      d = 1;
    else if (Iw < 0.5 * th_w && In < 0.5 * th_n)
      d = -1;
  } else {
    const double p = prob[b];
    d = p > 0.75 ? 1 : (p < 0.25 ? -1 : 0);
  }
  const int L = level[b];
  if (d > 0 && L >= max_level) d = 0;
  if (d < 0 && L == 0) d = 0;
  flags[b] = int8_t(d);
}

// ---- MLP ------------------------------------------------------------------------

constexpr int kMlpThreads = 256;

// Forward pass, one thread per sample; parameters staged in LDS.  Keeps
// h1 and h2 (pre-activation sign is h > 0) for the backward pass when asked.
__global__ void __launch_bounds__(kMlpThreads) mlp_forward_kernel(const float* params, const float* mean,
                                                                  const float* stdv, const float* X, int64_t n,
                                                                  float* prob, float* h1o, float* h2o) {
  __shared__ float P[kParams];
  for (int q = threadIdx.x; q < kParams; q += kMlpThreads) P[q] = params[q];
  __syncthreads();
  const int64_t b = int64_t(blockIdx.x) * kMlpThreads + threadIdx.x;
  if (b >= n) return;
  float x[kFeat];
  for (int k = 0; k < kFeat; ++k) x[k] = (X[b * kFeat + k] - mean[k]) / stdv[k];
  float h1[kHid];
  for (int j = 0; j < kHid; ++j) {
    float a = P[oB1 + j];
    for (int k = 0; k < kFeat; ++k) a += P[oW1 + j * kFeat + k] * x[k];
    h1[j] = fmaxf(a, 0.f);
    if (h1o) h1o[b * kHid + j] = h1[j];
  }
  float z = P[oB3];
  for (int j = 0; j < kHid; ++j) {
    float a = P[oB2 + j];
    for (int k = 0; k < kHid; ++k) a += P[oW2 + j * kHid + k] * h1[k];
    const float h2 = fmaxf(a, 0.f);
    if (h2o) h2o[b * kHid + j] = h2;
    z += P[oW3 + j] * h2;
  }
  prob[b] = 1.f / (1.f + expf(-z));
}

// dA2[b][j] = dz_b w3_j [h2 > 0], dz_b = (p_b - t_b) / B
__global__ void mlp_back2_kernel(const float* params, const float* prob, const float* target, const float* h2,
                                 int64_t n, float invB, float* dA2) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n * kHid) return;
  const int64_t b = q / kHid;
  const int j = int(q % kHid);
  const float dz = (prob[b] - target[b]) * invB;
  dA2[q] = h2[q] > 0.f ? dz * params[oW3 + j] : 0.f;
}

// dA1[b][k] = [h1 > 0] sum_j dA2[b][j] W2[j][k]
__global__ void mlp_back1_kernel(const float* params, const float* h1, const float* dA2, int64_t n, float* dA1) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n * kHid) return;
  const int64_t b = q / kHid;
  const int k = int(q % kHid);
  float s = 0.f;
  if (h1[q] > 0.f)
    for (int j = 0; j < kHid; ++j) s += dA2[b * kHid + j] * params[oW2 + j * kHid + k];
  dA1[q] = s;
}

// One thread per parameter: batch sums in a fixed order (deterministic).
__global__ void mlp_grad_kernel(const float* mean, const float* stdv, const float* X, const float* prob,
                                const float* target, const float* h1, const float* h2, const float* dA1,
                                const float* dA2, int64_t n, float invB, float* grad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kParams) return;
  float s = 0.f;
  if (q < oB1) {
    const int j = q / kFeat, k = q % kFeat;
    for (int64_t b = 0; b < n; ++b) s += dA1[b * kHid + j] * ((X[b * kFeat + k] - mean[k]) / stdv[k]);
  } else if (q < oW2) {
    const int j = q - oB1;
    for (int64_t b = 0; b < n; ++b) s += dA1[b * kHid + j];
  } else if (q < oB2) {
    const int j = (q - oW2) / kHid, k = (q - oW2) % kHid;
    for (int64_t b = 0; b < n; ++b) s += dA2[b * kHid + j] * h1[b * kHid + k];
  } else if (q < oW3) {
    const int j = q - oB2;
    for (int64_t b = 0; b < n; ++b) s += dA2[b * kHid + j];
  } else if (q < oB3) {
    const int j = q - oW3;
    for (int64_t b = 0; b < n; ++b) s += (prob[b] - target[b]) * invB * h2[b * kHid + j];
  } else {
    for (int64_t b = 0; b < n; ++b) s += (prob[b] - target[b]) * invB;
  }
  grad[q] = s;
}

__global__ void adam_kernel(float* params, float* m, float* v, const float* grad, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kParams) return;
  const float g = grad[q];
  m[q] = b1 * m[q] + (1.f - b1) * g;
  v[q] = b2 * v[q] + (1.f - b2) * g * g;
  params[q] -= lr * (m[q] / c1) / (sqrtf(v[q] / c2) + eps);
}

__global__ void gather_kernel(const float* X, const float* t, const int32_t* idx, int n, float* Xb, float* tb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int s = idx[q];
  for (int k = 0; k < kFeat; ++k) Xb[q * kFeat + k] = X[int64_t(s) * kFeat + k];
  tb[q] = t[s];
}

unsigned grid_of(int64_t n, int t) { return unsigned((n + t - 1) / t); }

uint64_t splitmix(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t& s) { return double(splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

// RAII device buffer list for the host entry points below.
struct Scratch {
  std::vector<void*> p;
  ~Scratch() {
    for (void* q : p) (void)hipFree(q);
  }
  template <typename T>
  hipError_t alloc(T** out, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) p.push_back(q);
    *out = static_cast<T*>(q);
    return e;
  }
};

}  // namespace

struct lbm_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  float* params = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* mean = nullptr;
  float* stdv = nullptr;
  std::vector<double> fmin, fmax;  // training range of the features
  int64_t adam_t = 0;
  ~lbm_mlp() {
    (void)hipSetDevice(device);
    for (float* q : {params, m, v, mean, stdv})
      if (q) (void)hipFree(q);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

// Forward (and optionally backward) over n samples already on the device.
int mlp_pass(lbm_mlp* m, Scratch& sc, const float* dX, const float* dt, int64_t n, float* dprob, float* dgrad) {
  float *h1 = nullptr, *h2 = nullptr;
  if (dgrad) {
    TRY(sc.alloc(&h1, size_t(n) * kHid));
    TRY(sc.alloc(&h2, size_t(n) * kHid));
  }
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid_of(n, kMlpThreads)), dim3(kMlpThreads), 0, m->stream, m->params,
                     m->mean, m->stdv, dX, n, dprob, h1, h2);
  TRY(hipGetLastError());
  if (!dgrad) return LBM_OK;
  float *dA1 = nullptr, *dA2 = nullptr;
  TRY(sc.alloc(&dA1, size_t(n) * kHid));
  TRY(sc.alloc(&dA2, size_t(n) * kHid));
  const float invB = 1.f / float(n);
  hipLaunchKernelGGL(mlp_back2_kernel, dim3(grid_of(n * kHid, 256)), dim3(256), 0, m->stream, m->params, dprob, dt,
                     h2, n, invB, dA2);
  hipLaunchKernelGGL(mlp_back1_kernel, dim3(grid_of(n * kHid, 256)), dim3(256), 0, m->stream, m->params, h1, dA2, n,
                     dA1);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(grid_of(kParams, 256)), dim3(256), 0, m->stream, m->mean, m->stdv, dX,
                     dprob, dt, h1, h2, dA1, dA2, n, invB, dgrad);
  TRY(hipGetLastError());
  return LBM_OK;
}

int upload_features(lbm_mlp* m, Scratch& sc, const double* X, int64_t n, float** dX) {
  std::vector<float> xf(size_t(n) * kFeat);
  for (size_t q = 0; q < xf.size(); ++q) xf[q] = float(X[q]);
  TRY(sc.alloc(dX, xf.size()));
  TRY(hipMemcpyAsync(*dX, xf.data(), xf.size() * sizeof(float), hipMemcpyHostToDevice, m->stream));
  TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

// Criterion values (and features) of the listed blocks of level L (all if
// `blocks` is null) with the two-pass cell / block kernels.
int criterion_level(lbm_forest* f, int L, const void* buf, const int32_t* blocks, int nblocks, double* drho,
                    double* u, double* neq, int64_t first, double* dfeat, double* dcrit) {
  const int n3 = f->n * f->n * f->n;
  const int64_t ncells = int64_t(nblocks) * n3;
  const unsigned g = grid_of(ncells, 256);
  switch (f->storage) {
    case LBM_F64:
      hipLaunchKernelGGL(cell_stats_kernel<double>, dim3(g), dim3(256), 0, f->stream, static_cast<const double*>(buf),
                         blocks, ncells, n3, drho, u, neq);
      break;
    case LBM_F32:
      hipLaunchKernelGGL(cell_stats_kernel<float>, dim3(g), dim3(256), 0, f->stream, static_cast<const float*>(buf),
                         blocks, ncells, n3, drho, u, neq);
      break;
    default:
      hipLaunchKernelGGL(cell_stats_kernel<__half>, dim3(g), dim3(256), 0, f->stream,
                         static_cast<const __half*>(buf), blocks, ncells, n3, drho, u, neq);
  }
  TRY(hipGetLastError());
  const int nlev = int(f->lv.size());
  hipLaunchKernelGGL(block_stats_kernel, dim3(nblocks), dim3(kStatThreads), 0, f->stream, drho, u, neq, f->n, blocks,
                     nblocks, double(L) / double(std::max(1, nlev - 1)), first, dfeat, dcrit);
  TRY(hipGetLastError());
  return LBM_OK;
}

// Features of every block (canonical order) in one fused pass per level.
int fused_features(lbm_forest* f, double* dfeat) {
  const int nlev = int(f->lv.size());
  int64_t first = 0;
  for (int L = 0; L < nlev; ++L) {
    const LevelDev& v = f->lv[L];
    if (!v.nblocks) continue;
    const double lf = double(L) / double(std::max(1, nlev - 1));
    const void* buf = current_state(f, L);
    switch (f->storage) {
      case LBM_F64:
        hipLaunchKernelGGL(block_features_kernel<double>, dim3(v.nblocks), dim3(kStatThreads), 0, f->stream,
                           static_cast<const double*>(buf), f->n, v.nblocks, lf, first, dfeat);
        break;
      case LBM_F32:
        hipLaunchKernelGGL(block_features_kernel<float>, dim3(v.nblocks), dim3(kStatThreads), 0, f->stream,
                           static_cast<const float*>(buf), f->n, v.nblocks, lf, first, dfeat);
        break;
      default:
        hipLaunchKernelGGL(block_features_kernel<__half>, dim3(v.nblocks), dim3(kStatThreads), 0, f->stream,
                           static_cast<const __half*>(buf), f->n, v.nblocks, lf, first, dfeat);
    }
    TRY(hipGetLastError());
    first += v.nblocks;
  }
  return LBM_OK;
}

__global__ void to_float_kernel(const double* x, int64_t n, float* y) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < n) y[q] = float(x[q]);
}

}  // namespace

extern "C" {

int lbm_plain_targets(const double* crit, int64_t n, double theta_omega, double theta_neq, double* target) {
  if ((!crit || !target) && n) return set_error(LBM_E_INVALID, "null pointer");
  for (int64_t b = 0; b < n; ++b) {
    const double Iw = crit[2 * b], In = crit[2 * b + 1];
    target[b] = (Iw > theta_omega || In > theta_neq) ? 1.0 : ((Iw < 0.5 * theta_omega && In < 0.5 * theta_neq) ? 0.0 : 0.5);
  }
  return LBM_OK;
}

int lbm_block_indicators(lbm_forest* f, double* features, double* crit) {
  if (!f || !features || !crit) return set_error(LBM_E_INVALID, "null pointer");
  TRY(hipSetDevice(f->device));
  if (int rc0 = prepare_state_read(f)) return rc0;
  int64_t nb = 0, maxcells = 0;
  for (const auto& v : f->lv) {
    nb += v.nblocks;
    maxcells = std::max<int64_t>(maxcells, v.ncells);
  }
  Scratch sc;
  double *drho, *u, *neq, *dfeat, *dcrit;
  TRY(sc.alloc(&drho, maxcells));
  TRY(sc.alloc(&u, 3 * maxcells));
  TRY(sc.alloc(&neq, maxcells));
  TRY(sc.alloc(&dfeat, nb * kFeat));
  TRY(sc.alloc(&dcrit, nb * 2));
  const int nlev = int(f->lv.size());
  int64_t first = 0;
  for (int L = 0; L < nlev; ++L) {
    const LevelDev& v = f->lv[L];
    if (!v.nblocks) continue;
    const void* buf = current_state(f, L);
    int rc = criterion_level(f, L, buf, nullptr, v.nblocks, drho, u, neq, first, dfeat, dcrit);
    if (rc) return rc;
    first += v.nblocks;
  }
  TRY(hipMemcpyAsync(features, dfeat, nb * kFeat * sizeof(double), hipMemcpyDeviceToHost, f->stream));
  TRY(hipMemcpyAsync(crit, dcrit, nb * 2 * sizeof(double), hipMemcpyDeviceToHost, f->stream));
  TRY(hipStreamSynchronize(f->stream));
  return LBM_OK;
}

int lbm_block_features(lbm_forest* f, double* features) {
  if (!f || !features) return set_error(LBM_E_INVALID, "null pointer");
  TRY(hipSetDevice(f->device));
  if (int rc0 = prepare_state_read(f)) return rc0;
  int64_t nb = 0;
  for (const auto& v : f->lv) nb += v.nblocks;
  Scratch sc;
  double* dfeat;
  TRY(sc.alloc(&dfeat, nb * kFeat));
  int rc = fused_features(f, dfeat);
  if (rc) return rc;
  TRY(hipMemcpyAsync(features, dfeat, nb * kFeat * sizeof(double), hipMemcpyDeviceToHost, f->stream));
  TRY(hipStreamSynchronize(f->stream));
  return LBM_OK;
}

int lbm_mlp_create(int device, uint64_t seed, lbm_mlp** out) {
  if (!out) return set_error(LBM_E_INVALID, "null pointer");
  *out = nullptr;
  TRY(hipSetDevice(device));
  lbm_mlp* m = new (std::nothrow) lbm_mlp();
  if (!m) return set_error(LBM_E_INVALID, "host allocation failed");
  m->device = device;
  auto body = [&]() -> int {
    TRY(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
    TRY(hipMalloc(&m->params, kParams * sizeof(float)));
    TRY(hipMalloc(&m->m, kParams * sizeof(float)));
    TRY(hipMalloc(&m->v, kParams * sizeof(float)));
    TRY(hipMalloc(&m->mean, kFeat * sizeof(float)));
    TRY(hipMalloc(&m->stdv, kFeat * sizeof(float)));
    // He initialisation (normal, Box-Muller on SplitMix64), zero biases
    std::vector<float> p(kParams, 0.f);
    uint64_t s = seed;
    auto normal = [&]() {
      const double u1 = std::max(uniform01(s), 1e-300), u2 = uniform01(s);
      return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    for (int q = 0; q < kHid * kFeat; ++q) p[oW1 + q] = float(normal() * std::sqrt(2.0 / kFeat));
    for (int q = 0; q < kHid * kHid; ++q) p[oW2 + q] = float(normal() * std::sqrt(2.0 / kHid));
    for (int q = 0; q < kHid; ++q) p[oW3 + q] = float(normal() * std::sqrt(1.0 / kHid));
    TRY(hipMemcpy(m->params, p.data(), kParams * sizeof(float), hipMemcpyHostToDevice));
    TRY(hipMemset(m->m, 0, kParams * sizeof(float)));
    TRY(hipMemset(m->v, 0, kParams * sizeof(float)));
    std::vector<float> zero(kFeat, 0.f), one(kFeat, 1.f);
    TRY(hipMemcpy(m->mean, zero.data(), kFeat * sizeof(float), hipMemcpyHostToDevice));
    TRY(hipMemcpy(m->stdv, one.data(), kFeat * sizeof(float), hipMemcpyHostToDevice));
    m->fmin.assign(kFeat, -1e300);
    m->fmax.assign(kFeat, 1e300);
    return LBM_OK;
  };
  int rc = body();
  if (rc) {
    delete m;
    return rc;
  }
  *out = m;
  return LBM_OK;
}

int lbm_mlp_destroy(lbm_mlp* m) {
  delete m;
  return LBM_OK;
}

int lbm_mlp_num_params(int* n) {
  if (!n) return set_error(LBM_E_INVALID, "null pointer");
  *n = kParams;
  return LBM_OK;
}

int lbm_mlp_get_params(lbm_mlp* m, float* params) {
  if (!m || !params) return set_error(LBM_E_INVALID, "null pointer");
  TRY(hipSetDevice(m->device));
  TRY(hipMemcpy(params, m->params, kParams * sizeof(float), hipMemcpyDeviceToHost));
  return LBM_OK;
}

int lbm_mlp_set_params(lbm_mlp* m, const float* params) {
  if (!m || !params) return set_error(LBM_E_INVALID, "null pointer");
  TRY(hipSetDevice(m->device));
  TRY(hipMemcpy(m->params, params, kParams * sizeof(float), hipMemcpyHostToDevice));
  TRY(hipMemset(m->m, 0, kParams * sizeof(float)));
  TRY(hipMemset(m->v, 0, kParams * sizeof(float)));
  m->adam_t = 0;
  return LBM_OK;
}

int lbm_mlp_set_normalization(lbm_mlp* m, const double* mean, const double* stdv, const double* fmin,
                              const double* fmax) {
  if (!m || !mean || !stdv) return set_error(LBM_E_INVALID, "null pointer");
  TRY(hipSetDevice(m->device));
  std::vector<float> a(kFeat), b(kFeat);
  for (int k = 0; k < kFeat; ++k) {
    if (!(stdv[k] > 0)) return set_error(LBM_E_INVALID, "std must be positive");
    a[k] = float(mean[k]);
    b[k] = float(stdv[k]);
  }
  TRY(hipMemcpy(m->mean, a.data(), kFeat * sizeof(float), hipMemcpyHostToDevice));
  TRY(hipMemcpy(m->stdv, b.data(), kFeat * sizeof(float), hipMemcpyHostToDevice));
  for (int k = 0; k < kFeat; ++k) {
    m->fmin[k] = fmin ? fmin[k] : -1e300;
    m->fmax[k] = fmax ? fmax[k] : 1e300;
  }
  return LBM_OK;
}

int lbm_mlp_predict(lbm_mlp* m, const double* X, int64_t n, float* prob) {
  if (!m || (!X && n) || (!prob && n) || n < 0) return set_error(LBM_E_INVALID, "bad arguments");
  if (!n) return LBM_OK;
  TRY(hipSetDevice(m->device));
  Scratch sc;
  float *dX, *dp;
  int rc = upload_features(m, sc, X, n, &dX);
  if (rc) return rc;
  TRY(sc.alloc(&dp, n));
  if ((rc = mlp_pass(m, sc, dX, nullptr, n, dp, nullptr))) return rc;
  TRY(hipMemcpyAsync(prob, dp, n * sizeof(float), hipMemcpyDeviceToHost, m->stream));
  TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

int lbm_mlp_gradient(lbm_mlp* m, const double* X, const double* target, int64_t n, float* grad) {
  if (!m || !X || !target || !grad || n <= 0) return set_error(LBM_E_INVALID, "bad arguments");
  TRY(hipSetDevice(m->device));
  Scratch sc;
  float *dX, *dt, *dp, *dg;
  int rc = upload_features(m, sc, X, n, &dX);
  if (rc) return rc;
  std::vector<float> tf(target, target + n);
  TRY(sc.alloc(&dt, n));
  TRY(sc.alloc(&dp, n));
  TRY(sc.alloc(&dg, kParams));
  TRY(hipMemcpyAsync(dt, tf.data(), n * sizeof(float), hipMemcpyHostToDevice, m->stream));
  if ((rc = mlp_pass(m, sc, dX, dt, n, dp, dg))) return rc;
  TRY(hipMemcpyAsync(grad, dg, kParams * sizeof(float), hipMemcpyDeviceToHost, m->stream));
  TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

int lbm_mlp_train(lbm_mlp* m, const double* X, const double* target, int64_t n, int epochs, int batch, double lr,
                  uint64_t seed, double* epoch_loss) {
  if (!m || !X || !target || n <= 0 || epochs < 0 || batch <= 0 || !(lr > 0))
    return set_error(LBM_E_INVALID, "bad arguments");
  TRY(hipSetDevice(m->device));
  Scratch sc;
  float *dX, *dt, *Xb, *tb, *pb, *gb, *pall;
  int32_t* didx;
  int rc = upload_features(m, sc, X, n, &dX);
  if (rc) return rc;
  std::vector<float> tf(target, target + n);
  TRY(sc.alloc(&dt, n));
  TRY(hipMemcpyAsync(dt, tf.data(), n * sizeof(float), hipMemcpyHostToDevice, m->stream));
  TRY(sc.alloc(&Xb, size_t(batch) * kFeat));
  TRY(sc.alloc(&tb, batch));
  TRY(sc.alloc(&pb, batch));
  TRY(sc.alloc(&gb, kParams));
  TRY(sc.alloc(&pall, n));
  TRY(sc.alloc(&didx, n));
  std::vector<int32_t> idx(n);
  for (int64_t q = 0; q < n; ++q) idx[q] = int32_t(q);
  uint64_t s = seed;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  std::vector<float> ph(n);
  for (int e = 0; e < epochs; ++e) {
    for (int64_t q = n - 1; q > 0; --q) std::swap(idx[q], idx[int64_t(splitmix(s) % uint64_t(q + 1))]);
    TRY(hipMemcpyAsync(didx, idx.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, m->stream));
    for (int64_t off = 0; off + batch <= n; off += batch) {
      hipLaunchKernelGGL(gather_kernel, dim3(grid_of(batch, 256)), dim3(256), 0, m->stream, dX, dt, didx + off, batch,
                         Xb, tb);
      Scratch step;
      if ((rc = mlp_pass(m, step, Xb, tb, batch, pb, gb))) return rc;
      m->adam_t++;
      const float c1 = 1.f - std::pow(b1, float(m->adam_t)), c2 = 1.f - std::pow(b2, float(m->adam_t));
      hipLaunchKernelGGL(adam_kernel, dim3(grid_of(kParams, 256)), dim3(256), 0, m->stream, m->params, m->m, m->v, gb,
                         float(lr), b1, b2, eps, c1, c2);
      TRY(hipGetLastError());
      TRY(hipStreamSynchronize(m->stream));  // `step` frees its buffers on scope exit
    }
    if (epoch_loss) {
      if ((rc = mlp_pass(m, sc, dX, nullptr, n, pall, nullptr))) return rc;
      TRY(hipMemcpyAsync(ph.data(), pall, n * sizeof(float), hipMemcpyDeviceToHost, m->stream));
      TRY(hipStreamSynchronize(m->stream));
      double l = 0;
      for (int64_t q = 0; q < n; ++q) {
        const double p = std::min(std::max(double(ph[q]), 1e-12), 1.0 - 1e-12);
        l -= target[q] * std::log(p) + (1.0 - target[q]) * std::log(1.0 - p);
      }
      epoch_loss[e] = l / double(n);
    }
  }
  TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

int lbm_mlp_fit_normalization(lbm_mlp* m, const double* X, int64_t n) {
  if (!m || !X || n < 2) return set_error(LBM_E_INVALID, "bad arguments");
  std::vector<double> mean(kFeat, 0.0), sd(kFeat, 0.0), lo(kFeat, 1e300), hi(kFeat, -1e300);
  for (int64_t b = 0; b < n; ++b)
    for (int k = 0; k < kFeat; ++k) {
      const double x = X[b * kFeat + k];
      mean[k] += x;
      lo[k] = std::min(lo[k], x);
      hi[k] = std::max(hi[k], x);
    }
  for (int k = 0; k < kFeat; ++k) mean[k] /= double(n);
  for (int64_t b = 0; b < n; ++b)
    for (int k = 0; k < kFeat; ++k) sd[k] += (X[b * kFeat + k] - mean[k]) * (X[b * kFeat + k] - mean[k]);
  for (int k = 0; k < kFeat; ++k) sd[k] = std::max(std::sqrt(sd[k] / double(n)), 1e-6);
  return lbm_mlp_set_normalization(m, mean.data(), sd.data(), lo.data(), hi.data());
}

int lbm_refinement_flags(lbm_forest* f, lbm_mlp* m, double theta_omega, double theta_neq, double delta,
                         int8_t* flags, int32_t* n_fallback) {
  if (!f || !flags) return set_error(LBM_E_INVALID, "null pointer");
  if (!(theta_omega > 0) || !(theta_neq > 0) || delta < 0) return set_error(LBM_E_INVALID, "bad thresholds");
  if (m && m->device != f->device) return set_error(LBM_E_INVALID, "MLP and forest on different devices");
  TRY(hipSetDevice(f->device));
  if (int rc0 = prepare_state_read(f)) return rc0;
  const int nlev = int(f->lv.size());
  int64_t nb = 0, maxcells = 0;
  std::vector<int64_t> first(nlev, 0);
  for (int L = 0; L < nlev; ++L) {
    first[L] = nb;
    nb += f->lv[L].nblocks;
    maxcells = std::max<int64_t>(maxcells, f->lv[L].ncells);
  }
  Scratch sc;
  double *dfeat, *dcrit, *drho, *du, *dneq;
  int32_t* dlev;
  int8_t *dflags, *dfb;
  float* dprob = nullptr;
  TRY(sc.alloc(&dfeat, nb * kFeat));
  TRY(sc.alloc(&dcrit, nb * 2));
  TRY(sc.alloc(&dlev, nb));
  TRY(sc.alloc(&dflags, nb));
  TRY(sc.alloc(&dfb, nb));
  std::vector<int32_t> lev;
  for (int L = 0; L < nlev; ++L) lev.insert(lev.end(), f->lv[L].nblocks, L);
  TRY(hipMemcpyAsync(dlev, lev.data(), lev.size() * sizeof(int32_t), hipMemcpyHostToDevice, f->stream));
  int rc;
  int32_t fallback = 0;
  if (!m) {
    TRY(sc.alloc(&drho, maxcells));
    TRY(sc.alloc(&du, 3 * maxcells));
    TRY(sc.alloc(&dneq, maxcells));
    for (int L = 0; L < nlev; ++L)
      if (f->lv[L].nblocks &&
          (rc = criterion_level(f, L, current_state(f, L), nullptr, f->lv[L].nblocks, drho, du, dneq, first[L], nullptr,
                                dcrit)))
        return rc;
  } else {
    // features in one pass, the MLP, then the criterion only where it decides
    if ((rc = fused_features(f, dfeat))) return rc;
    float* dX;
    double *dmin, *dmax;
    TRY(sc.alloc(&dX, nb * kFeat));
    TRY(sc.alloc(&dprob, nb));
    TRY(sc.alloc(&dmin, kFeat));
    TRY(sc.alloc(&dmax, kFeat));
    hipLaunchKernelGGL(to_float_kernel, dim3(grid_of(nb * kFeat, 256)), dim3(256), 0, f->stream, dfeat, nb * kFeat, dX);
    TRY(hipMemcpyAsync(dmin, m->fmin.data(), kFeat * sizeof(double), hipMemcpyHostToDevice, f->stream));
    TRY(hipMemcpyAsync(dmax, m->fmax.data(), kFeat * sizeof(double), hipMemcpyHostToDevice, f->stream));
    TRY(hipStreamSynchronize(f->stream));
    if ((rc = mlp_pass(m, sc, dX, nullptr, nb, dprob, nullptr))) return rc;
    TRY(hipStreamSynchronize(m->stream));
    hipLaunchKernelGGL(fallback_kernel, dim3(grid_of(nb, 256)), dim3(256), 0, f->stream, dfeat, dprob, dmin, dmax,
                       int(nb), delta, dfb);
    TRY(hipGetLastError());
    std::vector<int8_t> fb(nb);
    TRY(hipMemcpyAsync(fb.data(), dfb, nb, hipMemcpyDeviceToHost, f->stream));
    TRY(hipStreamSynchronize(f->stream));
    for (int64_t b = 0; b < nb; ++b) fallback += fb[b];
    if (fallback) {
      // per-cell buffers are indexed by the canonical cell index
      TRY(sc.alloc(&drho, maxcells));
      TRY(sc.alloc(&du, 3 * maxcells));
      TRY(sc.alloc(&dneq, maxcells));
    }
    for (int L = 0; L < nlev && fallback; ++L) {
      std::vector<int32_t> list;
      for (int b = 0; b < f->lv[L].nblocks; ++b)
        if (fb[first[L] + b]) list.push_back(b);
      if (list.empty()) continue;
      int32_t* dlist;
      TRY(sc.alloc(&dlist, list.size()));
      TRY(hipMemcpyAsync(dlist, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice, f->stream));
      if ((rc = criterion_level(f, L, current_state(f, L), dlist, int(list.size()), drho, du, dneq, first[L], nullptr,
                                dcrit)))
        return rc;
      TRY(hipStreamSynchronize(f->stream));
    }
  }
  hipLaunchKernelGGL(decide_kernel, dim3(grid_of(nb, 256)), dim3(256), 0, f->stream, dcrit, dprob, dfb, dlev, int(nb),
                     f->max_level, theta_omega, theta_neq, dflags);
  TRY(hipGetLastError());
  TRY(hipMemcpyAsync(flags, dflags, nb, hipMemcpyDeviceToHost, f->stream));
  TRY(hipStreamSynchronize(f->stream));
  if (n_fallback) *n_fallback = fallback;
  return LBM_OK;
}

}  // extern "C"
