// C ABI of the refined lattice Boltzmann library (declared in lbm_refined.h).
//
// Schedule of one coarse step (Algorithm 1 in post-collision form): the
// finer level's two substeps run before every substep of a level, so the
// launch list is the post-order of the level recursion,
//   sweep(Lmax, 1), sweep(Lmax, 2), sweep(Lmax - 1, 1), ..., sweep(0, 1),
// i.e. sum_L 2^L launches per coarse step.
//
// Buffers: level 0 alternates between two.  A level L >= 1 rotates through
// three: with its state at the start of a parent step in buffer r, the first
// substep writes r+1, the second reads r+1 and r and writes r+2 (mod 3); the
// coarser level then reads r (state at t) and r+1 (state at t + 1/2) for the
// coalescence.  The buffer assignment therefore repeats every 6 coarse steps;
// one graph is captured per distinct assignment.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <unordered_map>
#include <unordered_set>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm_refined.h"
#include "forest.hpp"
#include "inplace.hpp"
#include "kernels.hpp"
#include "state.hpp"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

namespace lbm {
int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
}  // namespace lbm

namespace {

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      if (e_ == hipErrorOutOfMemory) return fail(LBM_E_OOM, "%s: %s", #expr, hipGetErrorString(e_)); \
      return fail(LBM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));                        \
    }                                                                                        \
  } while (0)

}  // namespace

namespace {

template <typename T>
int dev_alloc(std::vector<void*>& owner, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return LBM_OK;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? LBM_E_OOM : LBM_E_HIP, "hipMalloc(%zu bytes): %s", count * sizeof(T),
                hipGetErrorString(e));
  }
  owner.push_back(q);
  *p = static_cast<T*>(q);
  return LBM_OK;
}

template <typename T>
int upload(std::vector<void*>& owner, T** p, const std::vector<T>& v) {
  int rc = dev_alloc(owner, p, v.size());
  if (rc) return rc;
  if (!v.empty()) HIP_TRY(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return LBM_OK;
}

// Device storage and tables of every level of `tabs`; buffers zeroed.
int make_levels(int n, size_t s, const std::vector<LevelTables>& tabs, std::vector<LevelDev>& lv) {
  const size_t n3 = size_t(n) * n * n;
  lv.assign(tabs.size(), LevelDev{});
  int rc;
  for (size_t L = 0; L < tabs.size(); ++L) {
    const LevelTables& t = tabs[L];
    LevelDev& v = lv[L];
    v.nblocks = t.nblocks;
    v.nwork = int(t.work.size());
    v.tiles_per_block = t.tiles_per_block;
    v.ncells = int64_t(t.nblocks) * int64_t(n3);
    v.plane = uint64_t(t.nblocks) * n3;
    if (v.plane >= (uint64_t(1) << 32))
      return fail(LBM_E_INVALID, "level %zu holds %llu cells; at most 2^32 - 1 per level are addressable", L,
                  (unsigned long long)v.plane);
    const size_t bytes = size_t(v.plane) * 19 * s;
    v.nbuf = L == 0 ? 2 : 3;
    const size_t fbytes = size_t(t.nblocks) * 10 * n * n * s;
    for (int b = 0; b < v.nbuf; ++b) {
      uint8_t* p = nullptr;
      if ((rc = dev_alloc(v.allocs, &p, bytes))) return rc;
      if (bytes) HIP_TRY(hipMemset(p, 0, bytes));
      v.buf[b] = p;
      p = nullptr;
      if ((rc = dev_alloc(v.allocs, &p, fbytes))) return rc;
      if (fbytes) HIP_TRY(hipMemset(p, 0, fbytes));
      v.xface[b] = p;
    }
    if ((rc = upload(v.allocs, &v.nbr, t.nbr))) return rc;
    if ((rc = upload(v.allocs, &v.flags, t.flags))) return rc;
    if ((rc = upload(v.allocs, &v.fine_index, t.fine_index))) return rc;
    if ((rc = upload(v.allocs, &v.fine_nbr, t.fine_nbr))) return rc;
    if ((rc = upload(v.allocs, &v.fine_slot, t.fine_slot))) return rc;
    if ((rc = upload(v.allocs, &v.cells, t.coal_cells))) return rc;
    if ((rc = upload(v.allocs, &v.chunks, t.coal_chunks))) return rc;
    v.nchunks = int32_t(t.coal_chunks.size() / 4);
    if (v.nchunks) {
      uint8_t* p = nullptr;
      if ((rc = dev_alloc(v.allocs, &p, size_t(t.fine_blocks) * 19 * n3 * s))) return rc;
      v.coal = p;
      if ((rc = dev_alloc(v.allocs, &p, size_t(t.fine_blocks) * 10 * n * n * s))) return rc;
      v.coal_x = p;
    }
    if ((rc = upload(v.allocs, &v.work, t.work))) return rc;
  }
  return LBM_OK;
}

void free_levels(std::vector<LevelDev>& lv) {
  for (auto& v : lv)
    for (void* p : v.allocs) (void)hipFree(p);
  lv.clear();
}

void set_level_omegas(lbm_forest* f);

// x-face copies of every level's current buffer, after the state was
// written by anything but a sweep (see CoalArgs).
int refresh_faces(lbm_forest* f) {
  for (size_t L = 0; L < f->lv.size(); ++L) {
    const LevelDev& v = f->lv[L];
    const int b = current_index(f, int(L));
    HIP_TRY(launch_face_copy(f->storage, f->n, v.buf[b], v.xface[b], v.nblocks, f->stream));
  }
  return LBM_OK;
}

void invalidate_graphs(lbm_forest* f) {
  for (auto& g : f->graphs) (void)hipGraphExecDestroy(g.second);
  f->graphs.clear();
}

// Post-order launch list: substep `substep` of level L, preceded by the two
// substeps of level L+1.  `r` holds every level's current buffer and is
// advanced as the launches are emitted.  parent_cur / parent_face: level
// L-1's state read by level L in this parent step, and its x-face copy.
void emit(const lbm_forest* f, int L, int substep, std::vector<int>& r, const void* parent_cur,
          const void* parent_face, std::vector<Op>& ops) {
  const LevelDev& d = f->lv[L];
  const int nlev = int(f->lv.size());
  const bool aa = f->inplace && f->inplace_level > 0 && L == f->inplace_level;  // refined, in place
  const void* prev = nullptr;
  int cb, nb;  // buffers read and written
  if (aa) {
    cb = nb = 0;
  } else if (L == 0) {
    cb = r[0];
    nb = r[0] ^ 1;
  } else if (substep == 1) {
    cb = r[L];
    nb = (r[L] + 1) % 3;
  } else {
    prev = d.buf[r[L]];
    cb = (r[L] + 1) % 3;
    nb = (r[L] + 2) % 3;
  }
  const void* cur = d.buf[cb];
  void* nxt = d.buf[nb];
  const void* fine0 = nullptr;
  const void* fine1 = nullptr;
  const void* fine0_x = nullptr;
  const void* fine1_x = nullptr;
  const void* save_t = nullptr;
  const void* save_half = nullptr;
  if (L + 1 < nlev) {
    const int rf = r[L + 1];
    emit(f, L + 1, 1, r, cur, d.xface[cb], ops);
    emit(f, L + 1, 2, r, cur, d.xface[cb], ops);
    const LevelDev& fd = f->lv[L + 1];
    if (f->inplace && L + 1 == f->inplace_level) {
      // the finer level in place: its states at t and t + 1/2 come from its saves
      fine0 = fine1 = fd.buf[0];
      fine0_x = fine1_x = fd.xface[0];
      save_t = f->save[rf];
      save_half = f->save[2];
    } else {
      fine0 = fd.buf[rf];
      fine1 = fd.buf[(rf + 1) % 3];
      fine0_x = fd.xface[rf];
      fine1_x = fd.xface[(rf + 1) % 3];
    }
  }
  Op op;
  op.level = L;
  SweepArgs& a = op.args;
  a.cur = cur;
  a.prev = prev;
  a.nxt = nxt;
  a.par = parent_cur;
  a.par_face = parent_face;
  a.fine0 = fine0;
  a.fine1 = fine1;
  a.work = nullptr;  // every tile of the level, in canonical order
  a.work0 = 0;
  a.nwork = d.nwork;
  a.xcd = d.order;
  a.substep = substep;
  a.collide = 1;
  a.nbr = d.nbr;
  a.flags = d.flags;
  a.fine_index = d.fine_index;
  a.coal = d.coal;
  a.coal_x = d.coal_x;
  a.face_cur = d.xface[cb];
  a.face_out = d.xface[nb];
  a.omega = float(d.omega);
  a.omega64 = d.omega;
  a.err = f->d_err;
  a.trt = f->trt ? 1 : 0;
  a.lambda_o = float(d.lambda_o);
  a.lambda_o64 = d.lambda_o;
  for (int q = 0; q < 3; ++q) {
    a.accel[q] = float(d.accel[q]);
    a.accel64[q] = d.accel[q];
  }
  a.interp = f->interp ? 1 : 0;
  a.par_nbr = L > 0 ? f->lv[L - 1].nbr : nullptr;
  a.fc = CoalArgs{};  // no coalescence in this launch (fuse_coalescence may add one)
  a.fc_stride = 0;
  if (L + 1 < nlev && d.nchunks > 0) {
    Op c;
    c.level = L;
    c.kind = Op::kCoalesce;
    c.args = a;
    c.coal.cur = cur;
    c.coal.fine0 = fine0;
    c.coal.fine1 = fine1;
    c.coal.out = d.coal;
    c.coal.out_x = d.coal_x;
    c.coal.fine0_x = fine0_x;
    c.coal.fine1_x = fine1_x;
    c.coal.cells = d.cells;
    c.coal.chunks = d.chunks;
    c.coal.nchunks = d.nchunks;
    c.coal.nbr = d.nbr;
    c.coal.fine_nbr = d.fine_nbr;
    c.coal.fine_slot = d.fine_slot;
    c.coal.check = f->coal_check ? f->d_check : nullptr;
    c.coal.err = f->d_err;
    c.coal.interp = f->interp ? 1 : 0;
    c.coal.walls = f->forest.periodic[0] && f->forest.periodic[1] && f->forest.periodic[2] ? 0 : 1;
    c.coal.save_t = save_t;
    c.coal.save_half = save_half;
    ops.push_back(c);
  }
  if (aa) {
    // the first substep is the odd launch, the second the even one; the
    // rotation entry is the parity q of the level's parent steps: saves at t
    // in save[q], at t + 1 into save[q ^ 1], at t + 1/2 in save[2]
    const int q = r[L] & 1;
    op.kind = Op::kInplace;
    op.odd = substep == 1 ? 1 : 0;
    InplaceArgs& ia = op.ia;
    ia = InplaceArgs{};
    ia.buf = d.buf[0];
    ia.face = d.xface[0];
    ia.entry = d.xface[1];
    ia.nbr = d.nbr;
    ia.nblocks = d.nblocks;
    ia.xcd = d.order;
    ia.trt = f->trt ? 1 : 0;
    ia.omega = float(d.omega);
    ia.omega64 = d.omega;
    ia.lambda_o = float(d.lambda_o);
    ia.lambda_o64 = d.lambda_o;
    for (int k = 0; k < 3; ++k) {
      ia.accel[k] = float(d.accel[k]);
      ia.accel64[k] = d.accel[k];
    }
    ia.refined = 1;
    ia.flags = d.flags;
    ia.par = parent_cur;
    ia.par_face = parent_face;
    ia.save_in = f->save[q];
    ia.save_out = substep == 1 ? f->save[2] : f->save[q ^ 1];
    ia.err = f->d_err;
  }
  ops.push_back(op);
  if (aa) {
    if (substep == 2) r[L] ^= 1;
  } else if (L == 0) {
    r[0] ^= 1;
  } else if (substep == 2) {
    r[L] = (r[L] + 2) % 3;
  }
}

int grid_for(const lbm_forest* f, int level, int nwork) {
  const int p = f->lv[level].persistent >= 0 ? f->lv[level].persistent : f->persistent;
  const int units = nwork * f->lv[level].split;
  if (p <= 0) return units;
  return std::max(1, std::min(units, f->num_cu * p));
}

// Moves each coalescence launch into the launch just before it, the finer
// level's second substep, where that is a sweep with one workgroup per work
// unit and the homogeneous explosion: its chunks then run while that sweep
// streams (SweepArgs::fc).  The chunks read the finer level's states at t
// and t + 1/2 and this level's current state, none of which the second
// substep writes, and they are done when the launch ends, before this
// level's sweep reads them.  Left as launches of their own: where the finer
// level's fusion is off (lbm_set_level_fusion; the autotuner picks it per
// level), on the per-block schedule, and where the finer level runs a
// persistent grid, the interpolated explosion or in place.
bool level_fuses(const lbm_forest* f, int L) { return f->lv[L].fuse >= 0 ? f->lv[L].fuse != 0 : f->fuse; }

void fuse_coalescence(const lbm_forest* f, std::vector<Op>& ops) {
  if (f->interp) return;
  std::vector<Op> out;
  out.reserve(ops.size());
  for (const Op& op : ops) {
    if (op.kind == Op::kCoalesce && !out.empty()) {
      Op& host = out.back();
      if (host.kind == Op::kSweep && host.level == op.level + 1 && host.args.substep == 2 && host.args.nwork > 0 &&
          host.args.fc.nchunks == 0 && level_fuses(f, host.level) &&
          grid_for(f, host.level, host.args.nwork) >= host.args.nwork * f->lv[host.level].split) {
        host.args.fc = op.coal;
        continue;
      }
    }
    out.push_back(op);
  }
  ops.swap(out);
}

hipError_t launch_level(const lbm_forest* f, const Op& op) {
  if (op.kind == Op::kInplace) return launch_inplace(f->storage, f->n, op.ia, op.odd != 0, f->stream);
  return launch_sweep(f->storage, f->n, op.args, grid_for(f, op.level, op.args.nwork), f->lv[op.level].split,
                      f->stream);
}

int run_ops(lbm_forest* f, const std::vector<Op>& ops, bool per_block) {
  for (const Op& op : ops) {
    if (op.kind == Op::kCoalesce) {
      HIP_TRY(launch_coalesce(f->storage, f->n, op.coal, f->stream));
      continue;
    }
    if (op.args.nwork <= 0) continue;
    if (!per_block || op.kind == Op::kInplace) {
      HIP_TRY(launch_level(f, op));
    } else {
      const LevelDev& d = f->lv[op.level];
      for (int s = 0; s < d.nblocks; ++s) {
        SweepArgs a = op.args;
        a.work = nullptr;
        a.work0 = s * d.tiles_per_block;
        a.nwork = d.tiles_per_block;
        HIP_TRY(launch_sweep(f->storage, f->n, a, a.nwork, 1, f->stream));
      }
    }
  }
  return LBM_OK;
}

int capture_graph(lbm_forest* f, const std::vector<Op>& ops, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(f->stream, hipStreamCaptureModeThreadLocal));
  int rc = run_ops(f, ops, false);
  hipError_t e = hipStreamEndCapture(f->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(LBM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(LBM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  return LBM_OK;
}

void set_level_omegas(lbm_forest* f) {
  for (size_t L = 0; L < f->lv.size(); ++L) {
    LevelDev& v = f->lv[L];
    const double p = std::ldexp(1.0, int(L));
    v.omega = 2.0 * f->omega0 / (2.0 * p + (1.0 - p) * f->omega0);  // eq. omega_scaling_0
    // TRT: lambda_e,L = omega_L, lambda_o,L by eq. lambda_oL; a_L by eq. force_scaling
    v.lambda_o = f->lambda_eo > 0.0 ? (4.0 - 2.0 * v.omega) / (2.0 + (4.0 * f->lambda_eo - 1.0) * v.omega) : v.omega;
    for (int d = 0; d < 3; ++d) v.accel[d] = f->accel0[d] / p;
  }
}

Accel level_accel(const lbm_forest* f, int L) {
  Accel a{{0.0, 0.0, 0.0}};
  if (f->trt)
    for (int d = 0; d < 3; ++d) a.a[d] = f->lv[L].accel[d];
  return a;
}

int check_err_flag(lbm_forest* f) {
  int h = 0;
  HIP_TRY(hipMemcpyAsync(&h, f->d_err, sizeof(int), hipMemcpyDeviceToHost, f->stream));
  HIP_TRY(hipStreamSynchronize(f->stream));
  if (h) return fail(LBM_E_STATE, "sweep table lookup failed (error bits 0x%x)", h);
  return LBM_OK;
}

const void* current_buffer(const lbm_forest* f, int L) { return f->lv[L].buf[current_index(f, L)]; }

// ---- in-place streaming (lbm_set_inplace; layouts in inplace.hpp) ----------

InplaceArgs inplace_args(const lbm_forest* f) {
  const LevelDev& v = f->lv[0];
  InplaceArgs a{};  // zeroed: refined = 0, no parent, no saves (a forest of one level)
  a.refined = 0;
  a.buf = v.buf[0];
  a.face = v.xface[0];
  a.entry = v.xface[1];  // the second x-face buffer serves as the entry buffer
  a.nbr = v.nbr;
  a.nblocks = v.nblocks;
  a.xcd = v.order;
  a.trt = f->trt ? 1 : 0;
  a.omega = float(v.omega);
  a.omega64 = v.omega;
  a.lambda_o = float(v.lambda_o);
  a.lambda_o64 = v.lambda_o;
  for (int d = 0; d < 3; ++d) {
    a.accel[d] = float(v.accel[d]);
    a.accel64[d] = v.accel[d];
  }
  return a;
}

// From the natural layout to the swapped one, with the x-face copy that the
// odd launch reads.
int inplace_begin(lbm_forest* f) {
  if (f->layout != kLayoutNatural) return LBM_OK;
  const int L = f->inplace_level;
  const LevelDev& v = f->lv[L];
  HIP_TRY(launch_face_copy(f->storage, f->n, v.buf[0], v.xface[0], v.nblocks, f->stream));
  if (L > 0)  // refined: the saves of the state at the start of the coming parent step
    HIP_TRY(launch_inplace_save_fill(f->storage, f->n, v.buf[0], f->save[f->rot[L] & 1], v.nbr, v.nblocks, f->stream));
  HIP_TRY(launch_inplace_swap(f->storage, f->n, v.buf[0], v.nblocks, f->stream));
  f->layout = kLayoutSwapped;
  return LBM_OK;
}

// One in-place coarse step: the odd launch from the swapped layout, the
// even one from the pushed layout.
int inplace_step(lbm_forest* f) {
  const bool odd = f->layout == kLayoutSwapped;
  if (f->schedule == LBM_SCHED_GRAPH) {
    const std::vector<int> key = {-1, odd ? 1 : 0};  // rotation keys are non-negative
    auto it = f->graphs.find(key);
    if (it == f->graphs.end()) {
      hipGraph_t g = nullptr;
      hipGraphExec_t ge = nullptr;
      HIP_TRY(hipStreamBeginCapture(f->stream, hipStreamCaptureModeThreadLocal));
      const hipError_t le = launch_inplace(f->storage, f->n, inplace_args(f), odd, f->stream);
      const hipError_t ce = hipStreamEndCapture(f->stream, &g);
      if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(LBM_E_HIP, "graph capture of the in-place launch: %s",
                    hipGetErrorString(le != hipSuccess ? le : ce));
      }
      const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) return fail(LBM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
      it = f->graphs.emplace(key, ge).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, f->stream));
  } else {
    HIP_TRY(launch_inplace(f->storage, f->n, inplace_args(f), odd, f->stream));
  }
  f->layout = odd ? kLayoutPushed : kLayoutSwapped;
  f->steps_since_state++;
  f->post_lost = true;
  return LBM_OK;
}

// Staging memory of lbm_get_moments_static: a file-scope device array, so
// that the call allocates nothing.  Each device holds its own copy, at an
// address that hipGetSymbolAddress gives once per device (the array's name
// is not a device address in host code).
constexpr int64_t kStageCells = int64_t(1) << 19;  // 524,288 cells per chunk: rho + u = 16 MiB
static __device__ __align__(256) double scratch[4 * kStageCells];
constexpr int kMaxDevices = 64;
std::mutex g_stage_mu;
double* g_stage[kMaxDevices] = {};

// The calling thread's current device must be `device`.
int moments_stage(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return fail(LBM_E_INVALID, "device ordinal %d out of range", device);
  std::lock_guard<std::mutex> lock(g_stage_mu);
  if (!g_stage[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(LBM_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_stage[device] = static_cast<double*>(p);
  }
  *out = g_stage[device];
  return LBM_OK;
}

void* current_buffer_mut(lbm_forest* f, int L) { return f->lv[L].buf[current_index(f, L)]; }

}  // namespace

int lbm::prepare_state_read(lbm_forest* f) {
  if (!f->inplace || f->layout == kLayoutNatural) return LBM_OK;
  const LevelDev& v = f->lv[f->inplace_level];
  // a refined forest's in-place level ends every coarse step swapped
  if (f->inplace_level > 0 && f->layout != kLayoutSwapped) return fail(LBM_E_STATE, "in-place layout out of step");
  if (f->layout == kLayoutPushed) {
    HIP_TRY(launch_inplace_entry_merge(f->storage, f->n, v.buf[0], v.xface[1], v.nblocks, f->stream));
    HIP_TRY(launch_inplace_pair_swap(f->storage, f->n, v.buf[0], v.nbr, v.nblocks, f->stream));
  }
  HIP_TRY(launch_inplace_swap(f->storage, f->n, v.buf[0], v.nblocks, f->stream));
  f->layout = kLayoutNatural;
  return LBM_OK;
}

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

int lbm_lattice(int32_t* e, double* w) {
  static const int E[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                               {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1},
                               {1, 0, -1}, {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  if (!e || !w) return fail(LBM_E_INVALID, "null pointer");
  for (int a = 0; a < 19; ++a) {
    for (int d = 0; d < 3; ++d) e[3 * a + d] = E[a][d];
    w[a] = a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  return LBM_OK;
}

static int validate_and_build(const lbm_forest_desc* d, Forest& forest, std::string& err) {
  const int n = d->cells_per_block;
  if (n != 4 && n != 8 && n != 16 && n != 32) {
    err = "cells_per_block must be 4, 8, 16 or 32";
    return LBM_E_INVALID;
  }
  for (int a = 0; a < 3; ++a)
    if (d->root_blocks[a] < 1 || d->root_blocks[a] > 4096) {
      err = "root_blocks out of range";
      return LBM_E_INVALID;
    }
  if (d->max_level < 0 || d->max_level > 20) {
    err = "max_level out of range";
    return LBM_E_INVALID;
  }
  if (d->storage != LBM_F64 && d->storage != LBM_F32 && d->storage != LBM_F16_SHIFTED) {
    err = "unknown storage form";
    return LBM_E_INVALID;
  }
  if (!d->leaves && d->num_leaves) {
    err = "num_leaves without leaves";
    return LBM_E_INVALID;
  }
  bool periodic[3];
  for (int a = 0; a < 3; ++a) {
    if (d->periodic[a] != 0 && d->periodic[a] != 1) {
      err = "periodic flags must be 0 or 1";
      return LBM_E_INVALID;
    }
    periodic[a] = d->periodic[a] != 0;
  }
  int rc;
  if (d->leaves) {
    rc = forest.build_from_leaves(d->root_blocks, n, periodic, d->leaves, d->num_leaves, d->balance != 0, err);
    if (rc == LBM_OK && forest.max_level > d->max_level) {
      err = "leaf level above max_level";
      return LBM_E_INVALID;
    }
    return rc;
  }
  return forest.build_from_callback(d->root_blocks, n, periodic, d->max_level, d->refine, d->refine_user, err);
}

int lbm_build_leaves(const lbm_forest_desc* d, int32_t* out, int64_t capacity, int64_t* count) {
  if (!d || !count) return fail(LBM_E_INVALID, "null pointer");
  Forest forest;
  std::string err;
  int rc = validate_and_build(d, forest, err);
  if (rc) return fail(rc, "%s", err.c_str());
  int64_t total = 0;
  for (int L = 0; L < forest.num_levels(); ++L) total += int64_t(forest.level_leaves(L).size());
  *count = total;
  if (!out) return LBM_OK;
  if (capacity < total) return fail(LBM_E_INVALID, "capacity %lld < %lld leaves", (long long)capacity, (long long)total);
  size_t k = 0;
  for (int L = 0; L < forest.num_levels(); ++L)
    for (const Leaf& l : forest.level_leaves(L)) {
      out[k++] = l.level;
      out[k++] = l.x;
      out[k++] = l.y;
      out[k++] = l.z;
    }
  return LBM_OK;
}

static void fill_stats(const LevelTables& t, int storage, int n, int64_t out[8]) {
  out[0] = t.nblocks;
  out[1] = t.coarse_blocks;
  out[2] = int64_t(t.nblocks) * n * n * n;
  out[3] = t.fine_blocks;
  out[4] = int64_t(t.work.size());
  out[5] = t.coalesced_pairs;
  out[6] = int64_t(storage_bytes(storage));
  out[7] = int64_t(n) * n * n;
}

int lbm_plan_level_stats(const lbm_forest_desc* d, int level, int64_t out[8]) {
  if (!d || !out) return fail(LBM_E_INVALID, "null pointer");
  Forest forest;
  std::vector<LevelTables> tabs;
  std::string err;
  int rc = validate_and_build(d, forest, err);
  if (rc) return fail(rc, "%s", err.c_str());
  rc = build_level_tables(forest, sweep_tile_cells(d->storage, d->cells_per_block), tabs, err);
  if (rc) return fail(rc, "%s", err.c_str());
  if (level < 0 || level >= int(tabs.size())) return fail(LBM_E_INVALID, "level out of range");
  fill_stats(tabs[level], d->storage, forest.n, out);
  return LBM_OK;
}

int lbm_create_block_forest(const lbm_forest_desc* d, lbm_forest** out) {
  if (!d || !out) return fail(LBM_E_INVALID, "null pointer");
  *out = nullptr;
  const int n = d->cells_per_block;
  std::unique_ptr<lbm_forest> f(new (std::nothrow) lbm_forest());
  if (!f) return fail(LBM_E_INVALID, "host allocation failed");
  f->storage = d->storage;
  f->n = n;
  f->device = d->device;
  std::string err;
  int rc = validate_and_build(d, f->forest, err);
  if (rc) return fail(rc, "%s", err.c_str());
  rc = build_level_tables(f->forest, sweep_tile_cells(f->storage, f->n), f->tabs, err);
  if (rc) return fail(rc, "%s", err.c_str());

  HIP_TRY(hipSetDevice(d->device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, d->device));
  f->num_cu = prop.multiProcessorCount;
  if (d->stream) {
    f->stream = static_cast<hipStream_t>(d->stream);
  } else {
    // graph capture needs a stream other than the legacy null stream
    HIP_TRY(hipStreamCreateWithFlags(&f->stream, hipStreamNonBlocking));
    f->own_stream = true;
  }

  const size_t s = storage_bytes(f->storage);
  f->max_level = d->max_level;
  if ((rc = make_levels(n, s, f->tabs, f->lv))) return rc;
  f->rot.assign(f->tabs.size(), 0);
  f->rot_prev = f->rot;
  if ((rc = dev_alloc(f->allocations, &f->d_err, 1))) return rc;
  HIP_TRY(hipMemset(f->d_err, 0, sizeof(int)));
  if ((rc = dev_alloc(f->allocations, &f->d_partials, size_t(kReduceGrid) * 5 * 21))) return rc;
  if ((rc = dev_alloc(f->allocations, &f->d_check, 3))) return rc;
  HIP_TRY(hipMemset(f->d_check, 0, 3 * sizeof(unsigned long long)));
  HIP_TRY(hipDeviceSynchronize());
  *out = f.release();
  g_err.clear();
  return LBM_OK;
}

int lbm_destroy(lbm_forest* f) {
  if (!f) return LBM_OK;
  (void)hipSetDevice(f->device);
  if (f->stream) (void)hipStreamSynchronize(f->stream);
  delete f;
  return LBM_OK;
}

int lbm_num_levels(const lbm_forest* f, int* num_levels) {
  if (!f || !num_levels) return fail(LBM_E_INVALID, "null pointer");
  *num_levels = int(f->lv.size());
  return LBM_OK;
}

int lbm_num_blocks(const lbm_forest* f, int level, int64_t* num_blocks) {
  if (!f || !num_blocks) return fail(LBM_E_INVALID, "null pointer");
  if (level < -1 || level >= int(f->lv.size())) return fail(LBM_E_INVALID, "level out of range");
  int64_t s = 0;
  for (int L = 0; L < int(f->lv.size()); ++L)
    if (level == -1 || level == L) s += f->lv[L].nblocks;
  *num_blocks = s;
  return LBM_OK;
}

int lbm_num_cells(const lbm_forest* f, int level, int64_t* num_cells) {
  if (!f || !num_cells) return fail(LBM_E_INVALID, "null pointer");
  if (level < -1 || level >= int(f->lv.size())) return fail(LBM_E_INVALID, "level out of range");
  int64_t s = 0;
  for (int L = 0; L < int(f->lv.size()); ++L)
    if (level == -1 || level == L) s += f->lv[L].ncells;
  *num_cells = s;
  return LBM_OK;
}

int lbm_get_leaves(const lbm_forest* f, int32_t* out) {
  if (!f || !out) return fail(LBM_E_INVALID, "null pointer");
  size_t k = 0;
  for (int L = 0; L < f->forest.num_levels(); ++L)
    for (const Leaf& l : f->forest.level_leaves(L)) {
      out[k++] = l.level;
      out[k++] = l.x;
      out[k++] = l.y;
      out[k++] = l.z;
    }
  return LBM_OK;
}

int lbm_level_stats(const lbm_forest* f, int level, int64_t out[8]) {
  if (!f || !out) return fail(LBM_E_INVALID, "null pointer");
  if (level < 0 || level >= int(f->lv.size())) return fail(LBM_E_INVALID, "level out of range");
  fill_stats(f->tabs[level], f->storage, f->n, out);
  return LBM_OK;
}

int lbm_set_level_omega(lbm_forest* f, double omega0) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  if (!(omega0 >= 0.0 && omega0 < 2.0)) return fail(LBM_E_INVALID, "omega0 must lie in [0, 2)");
  f->omega0 = omega0;
  set_level_omegas(f);
  f->omega_set = true;
  invalidate_graphs(f);
  return LBM_OK;
}

int lbm_set_trt_force(lbm_forest* f, double lambda_eo, const double* accel0) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  if (!(lambda_eo >= 0.0) || !std::isfinite(lambda_eo)) return fail(LBM_E_INVALID, "lambda_eo must be finite and >= 0");
  double a[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < 3 && accel0; ++d) {
    if (!std::isfinite(accel0[d])) return fail(LBM_E_INVALID, "acceleration must be finite");
    a[d] = accel0[d];
  }
  // the stored state is post-collision and holds the force term of one
  // collision: a new acceleration would leave it inconsistent
  if (f->state_set && (a[0] != f->accel0[0] || a[1] != f->accel0[1] || a[2] != f->accel0[2]))
    return fail(LBM_E_STATE, "the acceleration must be set before lbm_init_pdfs");
  f->lambda_eo = lambda_eo;
  for (int d = 0; d < 3; ++d) f->accel0[d] = a[d];
  f->trt = lambda_eo > 0.0 || a[0] != 0.0 || a[1] != 0.0 || a[2] != 0.0;
  set_level_omegas(f);
  invalidate_graphs(f);
  return LBM_OK;
}

int lbm_get_level_omega(const lbm_forest* f, int level, double* omega) {
  if (!f || !omega) return fail(LBM_E_INVALID, "null pointer");
  if (level < 0 || level >= int(f->lv.size())) return fail(LBM_E_INVALID, "level out of range");
  if (!f->omega_set) return fail(LBM_E_STATE, "omega not set");
  *omega = f->lv[level].omega;
  return LBM_OK;
}

int lbm_init_pdfs(lbm_forest* f, const double* rho, const double* u) {
  if (!f || !rho || !u) return fail(LBM_E_INVALID, "null pointer");
  HIP_TRY(hipSetDevice(f->device));
  int64_t total = 0;
  lbm_num_cells(f, -1, &total);
  double* d_rho = nullptr;
  double* d_u = nullptr;
  HIP_TRY(hipMalloc(&d_rho, std::max<int64_t>(total, 1) * sizeof(double)));
  hipError_t e = hipMalloc(&d_u, std::max<int64_t>(total, 1) * 3 * sizeof(double));
  if (e != hipSuccess) {
    (void)hipFree(d_rho);
    return fail(LBM_E_OOM, "hipMalloc: %s", hipGetErrorString(e));
  }
  int rc = LBM_OK;
  auto body = [&]() -> int {
    HIP_TRY(hipMemcpyAsync(d_rho, rho, total * sizeof(double), hipMemcpyHostToDevice, f->stream));
    HIP_TRY(hipMemcpyAsync(d_u, u, total * 3 * sizeof(double), hipMemcpyHostToDevice, f->stream));
    int64_t off = 0;
    std::fill(f->rot.begin(), f->rot.end(), 0);
    f->steps_since_state = 0;
    f->layout = kLayoutNatural;
    f->post_lost = false;
    for (size_t L = 0; L < f->lv.size(); ++L) {
      const LevelDev& v = f->lv[L];
      HIP_TRY(launch_init(f->storage, f->n, v.buf[0], d_rho + off, d_u + 3 * off, v.ncells, level_accel(f, int(L)),
                          f->stream));
      off += v.ncells;
    }
    int rc2 = refresh_faces(f);
    if (rc2) return rc2;
    HIP_TRY(hipStreamSynchronize(f->stream));
    f->state_set = true;
    return LBM_OK;
  };
  rc = body();
  (void)hipFree(d_rho);
  (void)hipFree(d_u);
  return rc;
}

namespace {
void release(std::vector<void*>& owner, void*& p) {
  if (!p) return;
  auto it = std::find(owner.begin(), owner.end(), p);
  if (it != owner.end()) owner.erase(it);
  (void)hipFree(p);
  p = nullptr;
}
}  // namespace

int lbm_set_inplace(lbm_forest* f, int on) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  if (on != 0 && on != 1) return fail(LBM_E_INVALID, "on must be 0 or 1");
  if ((on != 0) == f->inplace) return LBM_OK;
  HIP_TRY(hipSetDevice(f->device));
  const int Lf = int(f->lv.size()) - 1;  // the finest level streams in place
  LevelDev& v = f->lv[Lf];
  const size_t sb = storage_bytes(f->storage);
  const size_t save_bytes = size_t(v.nblocks) * size_t(kSaveArrayCount) * size_t(f->n) * size_t(f->n) * sb;
  if (on) {
    if (Lf > 0 && f->interp)
      return fail(LBM_E_STATE, "in-place streaming on a refined forest uses the homogeneous explosion");
    // the saves first, so that a failed allocation leaves the forest as it was
    void* saves[3] = {nullptr, nullptr, nullptr};
    if (Lf > 0) {
      for (int q = 0; q < 3; ++q) {
        uint8_t* p = nullptr;
        int rc = dev_alloc(v.allocs, &p, save_bytes);
        if (rc) {
          for (void*& r : saves) release(v.allocs, r);
          return rc;
        }
        saves[q] = p;
      }
    }
    // nothing queued may still use the buffers that are released
    HIP_TRY(hipStreamSynchronize(f->stream));
    const int c = f->rot[Lf];
    if (c != 0) {  // the current state into buffer 0
      std::swap(v.buf[0], v.buf[c]);
      std::swap(v.xface[0], v.xface[c]);
    }
    f->rot[Lf] = 0;
    f->rot_prev = f->rot;
    // the other PDF buffers go; one x-face buffer stays as the entry buffer
    for (int b = 1; b < v.nbuf; ++b) release(v.allocs, v.buf[b]);
    for (int b = 2; b < v.nbuf; ++b) release(v.allocs, v.xface[b]);
    for (int q = 0; q < 3; ++q) f->save[q] = saves[q];
    v.nbuf = 1;
    f->inplace = true;
    f->inplace_level = Lf;
    f->layout = kLayoutNatural;
  } else {
    int rc = prepare_state_read(f);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(f->stream));
    const int nbuf = Lf == 0 ? 2 : 3;
    // the buffers first, into temporaries: a failed allocation leaves in-place streaming on
    void* bufs[3] = {nullptr, nullptr, nullptr};
    void* faces[3] = {nullptr, nullptr, nullptr};
    for (int b = 1; b < nbuf && !rc; ++b) {
      uint8_t* p = nullptr;
      if ((rc = dev_alloc(v.allocs, &p, size_t(v.plane) * 19 * sb))) break;
      bufs[b] = p;
      if (b >= 2) {
        if ((rc = dev_alloc(v.allocs, &p, size_t(v.nblocks) * 10 * f->n * f->n * sb))) break;
        faces[b] = p;
      }
    }
    if (rc) {
      for (int b = 0; b < 3; ++b) {
        release(v.allocs, bufs[b]);
        release(v.allocs, faces[b]);
      }
      return rc;
    }
    for (int b = 1; b < nbuf; ++b) {
      v.buf[b] = bufs[b];
      if (b >= 2) v.xface[b] = faces[b];
    }
    for (int q = 0; q < 3; ++q) release(v.allocs, f->save[q]);
    v.nbuf = nbuf;
    f->rot[Lf] = 0;
    HIP_TRY(launch_face_copy(f->storage, f->n, v.buf[0], v.xface[0], v.nblocks, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
    f->inplace = false;
    f->inplace_level = 0;
    f->rot_prev = f->rot;
  }
  invalidate_graphs(f);
  return LBM_OK;
}

int lbm_device_memory(int device, int64_t* free_bytes, int64_t* total_bytes) {
  if (!free_bytes || !total_bytes) return fail(LBM_E_INVALID, "null pointer");
  HIP_TRY(hipSetDevice(device));
  size_t fr = 0, tot = 0;
  HIP_TRY(hipMemGetInfo(&fr, &tot));
  *free_bytes = int64_t(fr);
  *total_bytes = int64_t(tot);
  return LBM_OK;
}

int lbm_get_inplace(const lbm_forest* f, int* on) {
  if (!f || !on) return fail(LBM_E_INVALID, "null pointer");
  *on = f->inplace ? 1 : 0;
  return LBM_OK;
}

int lbm_set_explosion_interpolation(lbm_forest* f, int on) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  if (on && f->inplace && f->inplace_level > 0)
    return fail(LBM_E_STATE, "in-place streaming on a refined forest uses the homogeneous explosion");
  f->interp = on != 0;
  invalidate_graphs(f);
  return LBM_OK;
}

int lbm_set_coalescence_check(lbm_forest* f, int on) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  f->coal_check = on != 0;
  invalidate_graphs(f);
  return LBM_OK;
}

int lbm_set_coalescence_fusion(lbm_forest* f, int on) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  if (on != 0 && on != 1) return fail(LBM_E_INVALID, "on must be 0 or 1");
  f->fuse = on != 0;
  for (auto& v : f->lv) v.fuse = -1;
  invalidate_graphs(f);
  return LBM_OK;
}

int lbm_set_level_fusion(lbm_forest* f, int level, int on) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  if (level < 0 || level >= int(f->lv.size())) return fail(LBM_E_INVALID, "level out of range");
  if (on < -1 || on > 1) return fail(LBM_E_INVALID, "on must be -1, 0 or 1");
  f->lv[level].fuse = on;
  invalidate_graphs(f);
  return LBM_OK;
}

int lbm_get_level_fusion(const lbm_forest* f, int level, int* on) {
  if (!f || !on) return fail(LBM_E_INVALID, "null pointer");
  if (level < 0 || level >= int(f->lv.size())) return fail(LBM_E_INVALID, "level out of range");
  *on = level_fuses(f, level) ? 1 : 0;
  return LBM_OK;
}

int lbm_coalescence_check(lbm_forest* f, double out[3]) {
  if (!f || !out) return fail(LBM_E_INVALID, "null pointer");
  HIP_TRY(hipSetDevice(f->device));
  unsigned long long h[3];
  HIP_TRY(hipMemcpyAsync(h, f->d_check, sizeof h, hipMemcpyDeviceToHost, f->stream));
  HIP_TRY(hipMemsetAsync(f->d_check, 0, sizeof h, f->stream));
  HIP_TRY(hipStreamSynchronize(f->stream));
  double v[2];
  std::memcpy(v, h, sizeof v);
  out[0] = v[0];
  out[1] = v[1];
  out[2] = double(h[2]);
  return LBM_OK;
}

int lbm_set_schedule(lbm_forest* f, int schedule) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  if (schedule != LBM_SCHED_GRAPH && schedule != LBM_SCHED_DIRECT && schedule != LBM_SCHED_PER_BLOCK)
    return fail(LBM_E_INVALID, "unknown schedule");
  f->schedule = schedule;
  return LBM_OK;
}

int lbm_set_launch(lbm_forest* f, int persistent) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  if (persistent < 0 || persistent > 64) return fail(LBM_E_INVALID, "persistent must lie in [0, 64]");
  f->persistent = persistent;
  invalidate_graphs(f);
  return LBM_OK;
}

int lbm_set_level_launch(lbm_forest* f, int level, int persistent, int order, int split) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  if (level < 0 || level >= int(f->lv.size())) return fail(LBM_E_INVALID, "level out of range");
  if (persistent < -1 || persistent > 64) return fail(LBM_E_INVALID, "persistent must lie in [-1, 64]");
  if (order != 0 && order != 1) return fail(LBM_E_INVALID, "order must be 0 or 1");
  if (split != 1 && split != 2 && split != 4) return fail(LBM_E_INVALID, "split must be 1, 2 or 4");
  HIP_TRY(hipSetDevice(f->device));
  HIP_TRY(hipStreamSynchronize(f->stream));
  f->lv[level].persistent = persistent;
  f->lv[level].order = order;
  f->lv[level].split = sweep_split(f->storage, f->n, split);
  invalidate_graphs(f);
  return LBM_OK;
}

int lbm_get_level_launch(const lbm_forest* f, int level, int* persistent, int* order, int* split) {
  if (!f || !persistent || !order || !split) return fail(LBM_E_INVALID, "null pointer");
  if (level < 0 || level >= int(f->lv.size())) return fail(LBM_E_INVALID, "level out of range");
  *persistent = f->lv[level].persistent;
  *order = f->lv[level].order;
  *split = f->lv[level].split;
  return LBM_OK;
}

int lbm_autotune(lbm_forest* f, int n_steps, double* result) {
  if (!f || !result) return fail(LBM_E_INVALID, "null pointer");
  if (n_steps < 1) return fail(LBM_E_INVALID, "n_steps < 1");
  if (!f->omega_set) return fail(LBM_E_STATE, "lbm_set_level_omega must be called first");
  if (f->inplace) return fail(LBM_E_STATE, "the autotuner times the two-buffer sweep; switch in-place streaming off first");
  HIP_TRY(hipSetDevice(f->device));
  const int nl = int(f->lv.size());
  const size_t sb = storage_bytes(f->storage);
  // the tuning steps advance the state: keep every buffer and restore it;
  // copy[L][b] is null for a level without cells
  std::vector<void*> saved;  // owner of the copies
  std::vector<std::vector<uint8_t*>> copy(nl);
  auto cleanup = [&]() {
    for (void* p : saved) (void)hipFree(p);
  };
  const std::vector<int> rot = f->rot, rot_prev = f->rot_prev;
  const int64_t since = f->steps_since_state;
  auto body = [&]() -> int {
    int rc;
    for (int L = 0; L < nl; ++L) {
      const LevelDev& v = f->lv[L];
      const size_t bytes = size_t(v.plane) * 19 * sb;
      copy[L].assign(v.nbuf, nullptr);
      for (int b = 0; b < v.nbuf && bytes; ++b) {
        if ((rc = dev_alloc(saved, &copy[L][b], bytes))) return rc;
        HIP_TRY(hipMemcpyAsync(copy[L][b], v.buf[b], bytes, hipMemcpyDeviceToDevice, f->stream));
      }
    }
    // (persistent, order, split); splits the storage form does not allow
    // fall back to the largest allowed one
    static const int kCand[][3] = {{0, 0, 1}, {0, 1, 1}, {0, 0, 2}, {0, 1, 2}, {0, 0, 4}, {0, 1, 4}, {1, 0, 1},
                                   {1, 1, 1}, {2, 0, 1}, {2, 1, 1}, {4, 0, 1}, {4, 1, 1}, {8, 0, 1}, {8, 1, 1}};
    const int ncand = int(sizeof(kCand) / sizeof(kCand[0]));
    std::vector<double> best(nl, 1e300);
    std::vector<int> bp(nl, 0), bo(nl, 0), bs(nl, 1), bf(nl, 1);
    std::vector<double> ms(2 * nl), cms(nl);
    std::vector<int64_t> cnt(2 * nl), ccnt(nl);
    // two passes over the candidates, each candidate keeping its faster
    // pass: a drift of the clocks during the search then favours no candidate
    // every shape is timed with the coarser level's coalescence inside the
    // level's second substep (fuse 1) and in a launch of its own (fuse 0)
    for (int pass = 0; pass < 2; ++pass) {
      for (int c = 0; c < 2 * ncand; ++c) {
        const int* cand = kCand[c / 2];
        const int fz = 1 - c % 2;
        for (int L = 0; L < nl; ++L) {
          f->lv[L].persistent = cand[0];
          f->lv[L].order = cand[1];
          f->lv[L].split = sweep_split(f->storage, f->n, cand[2]);
          f->lv[L].fuse = fz;
        }
        if ((rc = lbm_time_launches(f, 1, ms.data(), cnt.data(), cms.data(), ccnt.data()))) return rc;  // warm-up
        if ((rc = lbm_time_launches(f, n_steps, ms.data(), cnt.data(), cms.data(), ccnt.data()))) return rc;
        for (int L = 0; L < nl; ++L) {
          // mean time of one step of level L: its substeps' mean launch
          // durations, plus the coarser level's coalescence where it runs as
          // a launch of its own (where level L's second substep runs it, the
          // substep's duration holds it)
          const double t = ms[2 * L] + (L > 0 ? ms[2 * L + 1] + (ccnt[L - 1] ? cms[L - 1] : 0.0) : 0.0);
          if (f->lv[L].nwork > 0 && t < best[L]) {
            best[L] = t;
            bp[L] = cand[0];
            bo[L] = cand[1];
            bs[L] = f->lv[L].split;
            bf[L] = fz;
          }
        }
      }
    }
    for (int L = 0; L < nl; ++L) {
      f->lv[L].persistent = bp[L];
      f->lv[L].order = bo[L];
      f->lv[L].split = bs[L];
      f->lv[L].fuse = bf[L];
      result[5 * L] = bp[L];
      result[5 * L + 1] = bo[L];
      result[5 * L + 2] = bs[L];
      result[5 * L + 3] = bf[L];
      result[5 * L + 4] = best[L] < 1e300 ? best[L] : 0.0;
    }
    for (int L = 0; L < nl; ++L) {
      const LevelDev& v = f->lv[L];
      const size_t bytes = size_t(v.plane) * 19 * sb;
      for (int b = 0; b < v.nbuf; ++b)
        if (copy[L][b]) HIP_TRY(hipMemcpyAsync(v.buf[b], copy[L][b], bytes, hipMemcpyDeviceToDevice, f->stream));
    }
    HIP_TRY(hipStreamSynchronize(f->stream));
    return LBM_OK;
  };
  int rc = body();
  f->rot = rot;
  f->rot_prev = rot_prev;
  f->steps_since_state = since;
  invalidate_graphs(f);
  if (!rc) rc = refresh_faces(f);  // the restored buffers' x-face copies
  if (!rc) {
    const hipError_t e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) rc = fail(LBM_E_HIP, "autotune: %s", hipGetErrorString(e));
  }
  cleanup();
  return rc;
}

int lbm_step_coarse(lbm_forest* f, int n_steps) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  if (n_steps < 0) return fail(LBM_E_INVALID, "n_steps < 0");
  if (!f->omega_set) return fail(LBM_E_STATE, "lbm_set_level_omega must be called first");
  HIP_TRY(hipSetDevice(f->device));
  if (f->inplace && f->inplace_level == 0) {
    int rc = n_steps > 0 ? inplace_begin(f) : LBM_OK;
    for (int s = 0; s < n_steps && !rc; ++s) rc = inplace_step(f);
    return rc;
  }
  if (f->inplace && n_steps > 0) {
    int rc = inplace_begin(f);
    if (rc) return rc;
  }
  for (int s = 0; s < n_steps; ++s) {
    std::vector<int> r = f->rot;
    std::vector<Op> ops;
    emit(f, 0, 1, r, nullptr, nullptr, ops);
    if (f->schedule != LBM_SCHED_PER_BLOCK) fuse_coalescence(f, ops);
    f->rot_prev = f->rot;
    f->steps_since_state++;
    f->post_lost = f->inplace;
    if (f->schedule == LBM_SCHED_GRAPH) {
      auto it = f->graphs.find(f->rot);
      if (it == f->graphs.end()) {
        hipGraphExec_t g = nullptr;
        int rc = capture_graph(f, ops, &g);
        if (rc) return rc;
        it = f->graphs.emplace(f->rot, g).first;
      }
      HIP_TRY(hipGraphLaunch(it->second, f->stream));
    } else {
      int rc = run_ops(f, ops, f->schedule == LBM_SCHED_PER_BLOCK);
      if (rc) return rc;
    }
    f->rot = r;
  }
  return LBM_OK;
}

int lbm_time_sweeps(lbm_forest* f, int n_steps, double* ms, int64_t* launches) {
  return lbm_time_launches(f, n_steps, ms, launches, nullptr, nullptr);
}

int lbm_time_launches(lbm_forest* f, int n_steps, double* ms, int64_t* launches, double* coal_ms,
                      int64_t* coal_launches) {
  if (!f || !ms || !launches || (!coal_ms) != (!coal_launches)) return fail(LBM_E_INVALID, "null pointer");
  if (n_steps < 1) return fail(LBM_E_INVALID, "n_steps < 1");
  if (!f->omega_set) return fail(LBM_E_STATE, "lbm_set_level_omega must be called first");
  HIP_TRY(hipSetDevice(f->device));
  const size_t nl = f->lv.size();
  // (slot, start event), the end event follows in `ends`; slot level * 2 + substep - 1 for a
  // sweep, 2 * levels + level for a coalescence
  std::vector<std::pair<size_t, hipEvent_t>> marks;
  std::vector<hipEvent_t> ends;
  auto cleanup = [&]() {
    for (auto& m : marks) (void)hipEventDestroy(m.second);
    for (auto& e : ends) (void)hipEventDestroy(e);
  };
  auto body = [&]() -> int {
    if (f->inplace && f->inplace_level > 0) {
      int rc = inplace_begin(f);
      if (rc) return rc;
    }
    if (f->inplace && f->inplace_level == 0) {
      // in-place streaming: the odd launch counts as substep 1, the even one as substep 2
      int rc = inplace_begin(f);
      if (rc) return rc;
      for (int s = 0; s < n_steps; ++s) {
        const bool odd = f->layout == kLayoutSwapped;
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        marks.emplace_back(odd ? 0 : 1, e0);
        HIP_TRY(hipEventCreate(&e1));
        ends.push_back(e1);
        HIP_TRY(hipEventRecord(e0, f->stream));
        HIP_TRY(launch_inplace(f->storage, f->n, inplace_args(f), odd, f->stream));
        HIP_TRY(hipEventRecord(e1, f->stream));
        f->layout = odd ? kLayoutPushed : kLayoutSwapped;
        f->steps_since_state++;
        f->post_lost = true;
      }
    }
    for (int s = 0; s < n_steps && !(f->inplace && f->inplace_level == 0); ++s) {
      std::vector<int> r = f->rot;
      std::vector<Op> ops;
      emit(f, 0, 1, r, nullptr, nullptr, ops);
      if (f->schedule != LBM_SCHED_PER_BLOCK) fuse_coalescence(f, ops);
      f->rot_prev = f->rot;
      f->steps_since_state++;
      f->post_lost = f->inplace;
      for (const Op& op : ops) {
        const bool coal = op.kind == Op::kCoalesce;
        if (!coal && op.args.nwork <= 0) continue;
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        marks.emplace_back(coal ? 2 * nl + size_t(op.level) : size_t(op.level) * 2 + size_t(op.args.substep - 1), e0);
        HIP_TRY(hipEventCreate(&e1));
        ends.push_back(e1);
        HIP_TRY(hipEventRecord(e0, f->stream));
        if (coal)
          HIP_TRY(launch_coalesce(f->storage, f->n, op.coal, f->stream));
        else
          HIP_TRY(launch_level(f, op));
        HIP_TRY(hipEventRecord(e1, f->stream));
      }
      f->rot = r;
    }
    HIP_TRY(hipStreamSynchronize(f->stream));
    std::vector<double> tsum(3 * nl, 0.0);
    std::vector<int64_t> tcnt(3 * nl, 0);
    for (size_t i = 0; i < marks.size(); ++i) {
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, marks[i].second, ends[i]));
      tsum[marks[i].first] += t;
      tcnt[marks[i].first] += 1;
    }
    for (size_t i = 0; i < 3 * nl; ++i) {
      const double mean = tcnt[i] ? tsum[i] / double(tcnt[i]) : 0.0;
      if (i < 2 * nl) {
        ms[i] = mean;
        launches[i] = tcnt[i];
      } else if (coal_ms) {
        coal_ms[i - 2 * nl] = mean;
        coal_launches[i - 2 * nl] = tcnt[i];
      }
    }
    return LBM_OK;
  };
  int rc = body();
  cleanup();
  return rc;
}

int lbm_regrid(lbm_forest* f, const int8_t* flags, int64_t count) {
  if (!f || (!flags && count)) return fail(LBM_E_INVALID, "null pointer");
  if (f->inplace || f->post_lost)
    return fail(LBM_E_STATE,
                "regrid needs the state at the start of the last coarse step, which in-place streaming does not "
                "keep: switch it off and take a coarse step first");
  if (f->trt) return fail(LBM_E_STATE, "regrid supports the SRT collision without a body force");
  HIP_TRY(hipSetDevice(f->device));
  int rc = check_err_flag(f);
  if (rc) return rc;
  std::string err;
  Forest nf;
  if ((rc = f->forest.regrid(flags, count, f->max_level, nf, err))) return fail(rc, "%s", err.c_str());
  std::vector<LevelTables> ntabs;
  if ((rc = build_level_tables(nf, sweep_tile_cells(f->storage, f->n), ntabs, err))) return fail(rc, "%s", err.c_str());

  const int n = f->n;
  const size_t n3 = size_t(n) * n * n;
  const size_t sb = storage_bytes(f->storage);
  const int nold = int(f->lv.size());
  // old leaves by key
  std::unordered_map<uint64_t, std::pair<int, int>> old_slot;
  for (int L = 0; L < nold; ++L) {
    const auto& lv = f->forest.level_leaves(L);
    for (int b = 0; b < int(lv.size()); ++b) old_slot[block_key(L, lv[b].x, lv[b].y, lv[b].z)] = {L, b};
  }
  std::unordered_set<uint64_t> new_keys;
  for (int L = 0; L < nf.num_levels(); ++L)
    for (const Leaf& l : nf.level_leaves(L)) new_keys.insert(block_key(L, l.x, l.y, l.z));

  std::vector<void*> scratch;  // freed on every exit path below
  auto cleanup = [&]() {
    for (void* p : scratch) (void)hipFree(p);
  };
  auto body = [&]() -> int {
    // post-streaming values of the old blocks that change (section 4: the
    // state between coarse steps is post-streaming): re-run each level's
    // last launch of the last coarse step without the collision, into a
    // scratch buffer; its inputs are still intact
    const bool have_post = f->steps_since_state > 0;
    std::vector<const void*> post(nold, nullptr), cur(nold, nullptr);
    std::vector<uint64_t> planes(nold, 0);
    std::vector<Op> ops;
    if (have_post) {
      std::vector<int> r = f->rot_prev;
      emit(f, 0, 1, r, nullptr, nullptr, ops);
    }
    for (int L = 0; L < nold; ++L) {
      cur[L] = current_buffer(f, L);
      planes[L] = f->lv[L].plane;
      post[L] = cur[L];
      if (!have_post) continue;
      std::vector<int32_t> work;
      const auto& lv = f->forest.level_leaves(L);
      const int tpb = f->lv[L].tiles_per_block;
      for (int b = 0; b < int(lv.size()); ++b)
        if (!new_keys.count(block_key(L, lv[b].x, lv[b].y, lv[b].z)))
          for (int t = 0; t < tpb; ++t) work.push_back(b * tpb + t);
      if (work.empty()) continue;
      const Op* last = nullptr;
      const Op* last_coal = nullptr;
      for (const Op& op : ops)
        if (op.level == L) (op.kind == Op::kCoalesce ? last_coal : last) = &op;
      if (!last) return fail(LBM_E_STATE, "no launch recorded for level %d", L);
      // the coalesced values of that launch, recomputed from the same buffers
      if (last_coal) HIP_TRY(launch_coalesce(f->storage, n, last_coal->coal, f->stream));
      uint8_t* tmp = nullptr;
      int32_t* dwork = nullptr;
      int rc2;
      if ((rc2 = dev_alloc(scratch, &tmp, size_t(planes[L]) * 19 * sb))) return rc2;
      if ((rc2 = upload(scratch, &dwork, work))) return rc2;
      SweepArgs a = last->args;
      a.nxt = tmp;
      a.face_out = nullptr;
      a.collide = 0;
      a.work = dwork;
      a.nwork = int32_t(work.size());
      HIP_TRY(launch_sweep(f->storage, n, a, a.nwork, 1, f->stream));
      post[L] = tmp;
    }
    const void** d_cur = nullptr;
    const void** d_post = nullptr;
    int rc2;
    if ((rc2 = upload(scratch, &d_cur, cur))) return rc2;
    if ((rc2 = upload(scratch, &d_post, post))) return rc2;

    std::vector<LevelDev> nlv;
    if ((rc2 = make_levels(n, sb, ntabs, nlv))) {
      free_levels(nlv);
      return rc2;
    }
    for (int L = 0; L < int(ntabs.size()); ++L) {
      const auto& lv = nf.level_leaves(L);
      std::vector<RemapBlock> rb(lv.size());
      for (size_t b = 0; b < lv.size(); ++b) {
        const Leaf& l = lv[b];
        RemapBlock& e = rb[b];
        std::fill(e.slot, e.slot + 8, 0);
        e.off[0] = e.off[1] = e.off[2] = 0;
        e.shift = 0;
        auto it = old_slot.find(block_key(L, l.x, l.y, l.z));
        if (it != old_slot.end()) {
          e.mode = 0;
          e.src_level = L;
          e.slot[0] = it->second.second;
          continue;
        }
        bool found = false;
        for (int up = 1; up <= L && !found; ++up) {
          auto a = old_slot.find(block_key(L - up, l.x >> up, l.y >> up, l.z >> up));
          if (a == old_slot.end()) continue;
          e.mode = 1;
          e.src_level = L - up;
          e.shift = up;
          e.slot[0] = a->second.second;
          e.off[0] = ((l.x * n) >> up) - (l.x >> up) * n;
          e.off[1] = ((l.y * n) >> up) - (l.y >> up) * n;
          e.off[2] = ((l.z * n) >> up) - (l.z >> up) * n;
          found = true;
        }
        if (found) continue;
        e.mode = 2;
        e.src_level = L + 1;
        for (int o = 0; o < 8; ++o) {
          auto c = old_slot.find(block_key(L + 1, 2 * l.x + (o & 1), 2 * l.y + ((o >> 1) & 1), 2 * l.z + (o >> 2)));
          if (c == old_slot.end()) {
            free_levels(nlv);
            return fail(LBM_E_STATE, "regrid: block (%d,%d,%d,%d) has no source", L, l.x, l.y, l.z);
          }
          e.slot[o] = c->second.second;
        }
      }
      RemapBlock* d_rb = nullptr;
      if ((rc2 = upload(scratch, &d_rb, rb))) {
        free_levels(nlv);
        return rc2;
      }
      RemapArgs ra;
      ra.dst = nlv[L].buf[0];
      ra.blocks = d_rb;
      ra.ncells = int64_t(lv.size()) * int64_t(n3);
      ra.old_cur = d_cur;
      ra.old_post = d_post;
      ra.collide = have_post ? 1 : 0;
      const double p2 = std::ldexp(1.0, L);
      ra.omega64 = 2.0 * f->omega0 / (2.0 * p2 + (1.0 - p2) * f->omega0);
      ra.omega = float(ra.omega64);
      hipError_t e = launch_remap(f->storage, n, ra, f->stream);
      if (e != hipSuccess) {
        free_levels(nlv);
        return fail(LBM_E_HIP, "remap: %s", hipGetErrorString(e));
      }
    }
    hipError_t e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) {
      free_levels(nlv);
      return fail(LBM_E_HIP, "regrid: %s", hipGetErrorString(e));
    }
    invalidate_graphs(f);
    for (size_t L = 0; L < nlv.size() && L < f->lv.size(); ++L) {
      nlv[L].persistent = f->lv[L].persistent;
      nlv[L].order = f->lv[L].order;
      nlv[L].split = f->lv[L].split;
      nlv[L].fuse = f->lv[L].fuse;
    }
    free_levels(f->lv);
    f->lv = std::move(nlv);
    f->tabs = std::move(ntabs);
    f->forest = std::move(nf);
    f->rot.assign(f->lv.size(), 0);
    f->rot_prev = f->rot;
    f->steps_since_state = 0;
    set_level_omegas(f);
    return refresh_faces(f);
  };
  rc = body();
  cleanup();
  return rc;
}

int lbm_synchronize(lbm_forest* f) {
  if (!f) return fail(LBM_E_INVALID, "null pointer");
  HIP_TRY(hipSetDevice(f->device));
  HIP_TRY(hipStreamSynchronize(f->stream));
  return LBM_OK;
}

int lbm_get_moments(lbm_forest* f, double* rho, double* u) {
  if (!f || !rho || !u) return fail(LBM_E_INVALID, "null pointer");
  HIP_TRY(hipSetDevice(f->device));
  int rc = check_err_flag(f);
  if (rc) return rc;
  if ((rc = prepare_state_read(f))) return rc;
  int64_t off = 0;
  for (size_t L = 0; L < f->lv.size(); ++L) {
    const LevelDev& v = f->lv[L];
    if (v.ncells == 0) continue;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, v.ncells * 4 * sizeof(double)));
    auto body = [&]() -> int {
      HIP_TRY(launch_moments(f->storage, f->n, current_buffer(f, int(L)), d, d + v.ncells, 0, v.ncells,
                             level_accel(f, int(L)), f->stream));
      HIP_TRY(hipMemcpyAsync(rho + off, d, v.ncells * sizeof(double), hipMemcpyDeviceToHost, f->stream));
      HIP_TRY(hipMemcpyAsync(u + 3 * off, d + v.ncells, v.ncells * 3 * sizeof(double), hipMemcpyDeviceToHost,
                             f->stream));
      HIP_TRY(hipStreamSynchronize(f->stream));
      return LBM_OK;
    };
    rc = body();
    (void)hipFree(d);
    if (rc) return rc;
    off += v.ncells;
  }
  return LBM_OK;
}

int lbm_get_moments_static(lbm_forest* f, double* rho, double* u) {
  if (!f || !rho || !u) return fail(LBM_E_INVALID, "null pointer");
  HIP_TRY(hipSetDevice(f->device));
  double* stage = nullptr;
  int rc = moments_stage(f->device, &stage);
  if (rc) return rc;
  if ((rc = check_err_flag(f))) return rc;
  if ((rc = prepare_state_read(f))) return rc;
  int64_t off = 0;
  for (size_t L = 0; L < f->lv.size(); ++L) {
    const LevelDev& v = f->lv[L];
    // chunks of at most kStageCells cells: rho in stage[0, kStageCells),
    // u in stage[kStageCells, 4 kStageCells); the stream orders each chunk's
    // copies before the next chunk's kernel overwrites the stage
    for (int64_t c0 = 0; c0 < v.ncells; c0 += kStageCells) {
      const int64_t m = std::min<int64_t>(kStageCells, v.ncells - c0);
      HIP_TRY(launch_moments(f->storage, f->n, current_buffer(f, int(L)), stage, stage + kStageCells, c0, m,
                             level_accel(f, int(L)), f->stream));
      HIP_TRY(hipMemcpyAsync(rho + off + c0, stage, m * sizeof(double), hipMemcpyDeviceToHost, f->stream));
      HIP_TRY(hipMemcpyAsync(u + 3 * (off + c0), stage + kStageCells, m * 3 * sizeof(double), hipMemcpyDeviceToHost,
                             f->stream));
    }
    off += v.ncells;
  }
  HIP_TRY(hipStreamSynchronize(f->stream));
  return LBM_OK;
}

int lbm_get_pdfs(lbm_forest* f, double* h) {
  if (!f || !h) return fail(LBM_E_INVALID, "null pointer");
  HIP_TRY(hipSetDevice(f->device));
  if (int rc = prepare_state_read(f)) return rc;
  int64_t off = 0;
  for (size_t L = 0; L < f->lv.size(); ++L) {
    const LevelDev& v = f->lv[L];
    if (v.ncells == 0) continue;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, v.ncells * 19 * sizeof(double)));
    auto body = [&]() -> int {
      HIP_TRY(launch_get_pdfs(f->storage, f->n, current_buffer(f, int(L)), d, v.ncells, f->stream));
      HIP_TRY(hipMemcpyAsync(h + 19 * off, d, v.ncells * 19 * sizeof(double), hipMemcpyDeviceToHost, f->stream));
      HIP_TRY(hipStreamSynchronize(f->stream));
      return LBM_OK;
    };
    int rc = body();
    (void)hipFree(d);
    if (rc) return rc;
    off += v.ncells;
  }
  return LBM_OK;
}

int lbm_set_pdfs(lbm_forest* f, const double* h) {
  if (!f || !h) return fail(LBM_E_INVALID, "null pointer");
  HIP_TRY(hipSetDevice(f->device));
  int64_t off = 0;
  for (size_t L = 0; L < f->lv.size(); ++L) {
    const LevelDev& v = f->lv[L];
    if (v.ncells == 0) continue;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, v.ncells * 19 * sizeof(double)));
    auto body = [&]() -> int {
      HIP_TRY(hipMemcpyAsync(d, h + 19 * off, v.ncells * 19 * sizeof(double), hipMemcpyHostToDevice, f->stream));
      HIP_TRY(launch_set_pdfs(f->storage, f->n, current_buffer_mut(f, int(L)), d, v.ncells, f->stream));
      f->steps_since_state = 0;
      f->state_set = true;
      f->layout = kLayoutNatural;
      f->post_lost = false;
      HIP_TRY(launch_face_copy(f->storage, f->n, current_buffer(f, int(L)), v.xface[current_index(f, int(L))], v.nblocks,
                               f->stream));
      HIP_TRY(hipStreamSynchronize(f->stream));
      return LBM_OK;
    };
    int rc = body();
    (void)hipFree(d);
    if (rc) return rc;
    off += v.ncells;
  }
  return LBM_OK;
}

int lbm_mass(lbm_forest* f, double* mass, double momentum[3]) {
  if (!f || !mass || !momentum) return fail(LBM_E_INVALID, "null pointer");
  HIP_TRY(hipSetDevice(f->device));
  int rc = check_err_flag(f);
  if (rc) return rc;
  if ((rc = prepare_state_read(f))) return rc;
  const size_t nl = f->lv.size();
  for (size_t L = 0; L < nl; ++L) {
    if (f->lv[L].ncells == 0) continue;
    HIP_TRY(launch_reduce(f->storage, f->n, current_buffer(f, int(L)), f->lv[L].ncells,
                          f->d_partials + L * kReduceGrid * 5, f->stream));
  }
  std::vector<double> part(nl * kReduceGrid * 5, 0.0);
  for (size_t L = 0; L < nl; ++L) {
    if (f->lv[L].ncells == 0) continue;
    HIP_TRY(hipMemcpyAsync(part.data() + L * kReduceGrid * 5, f->d_partials + L * kReduceGrid * 5,
                           kReduceGrid * 5 * sizeof(double), hipMemcpyDeviceToHost, f->stream));
  }
  HIP_TRY(hipStreamSynchronize(f->stream));
  double M = 0, J[3] = {0, 0, 0}, bad = 0;
  for (size_t L = 0; L < nl; ++L) {
    if (f->lv[L].ncells == 0) continue;
    double s[5] = {0, 0, 0, 0, 0};
    for (int b = 0; b < kReduceGrid; ++b)
      for (int c = 0; c < 5; ++c) s[c] += part[(L * kReduceGrid + b) * 5 + c];
    const double w = std::ldexp(1.0, -3 * int(L));  // cell volume (dx_L / dx_0)^3
    M += w * (double(f->lv[L].ncells) + s[0]);      // sum_a f_a = 1 + sum_a h_a per cell
    for (int c = 0; c < 3; ++c) J[c] += w * s[1 + c];
    bad += s[4];
  }
  *mass = M;
  for (int c = 0; c < 3; ++c) momentum[c] = J[c];
  if (bad != 0 || !std::isfinite(M) || !std::isfinite(J[0]) || !std::isfinite(J[1]) || !std::isfinite(J[2]))
    return fail(LBM_E_NONFINITE, "NaN or Inf in the PDFs");
  return LBM_OK;
}

}  // extern "C"
