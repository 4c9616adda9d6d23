// Internal state of a forest handle, shared by the library's C ABI units.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <vector>

#include "../../include/lbm_refined.h"
#include "forest.hpp"
#include "inplace.hpp"
#include "kernels.hpp"

namespace lbm {

inline size_t storage_bytes(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32 ? 4 : 2); }


struct LevelDev {
  int64_t ncells = 0;  // interior cells
  uint64_t plane = 0;  // cells per direction: blocks * n^3 (a buffer holds 19 plane elements)
  int nblocks = 0, nwork = 0, tiles_per_block = 0;
  int nbuf = 0;
  void* buf[3] = {nullptr, nullptr, nullptr};
  int32_t* nbr = nullptr;
  uint32_t* flags = nullptr;
  int32_t* fine_index = nullptr;
  int32_t* fine_nbr = nullptr;
  int32_t* fine_slot = nullptr;
  uint16_t* cells = nullptr;    // cells of the coalesced pairs
  int32_t* chunks = nullptr;    // coalescence work: fine_nbr row, slot, first pair, count | direction << 16
  int32_t nchunks = 0;
  void* coal = nullptr;         // coalesced values [fine row][19][n^3]
  void* coal_x = nullptr;       // coalesced values of x-crossing pairs [fine row][10][n^2]
  void* xface[3] = {nullptr, nullptr, nullptr};  // x-face copy of each buffer [slot][10][n^2]
  int32_t* work = nullptr;      // work tiles in canonical order
  int persistent = -1;          // launch shape of this level; -1: the forest-wide setting
  int fuse = -1;                // 1: its second substep runs level L-1's coalescence (0 not; -1 forest-wide)
  int order = 0;                // 0 canonical unit order, 1 XCD-grouped (SweepArgs::xcd)
  int split = 1;                // workgroups per work tile (1, 2 or 4; see sweep_split)
  double omega = 0.0;           // omega_L (SRT) or lambda_e,L (TRT)
  double lambda_o = 0.0;        // lambda_o,L (TRT)
  double accel[3] = {0.0, 0.0, 0.0};  // lattice acceleration a_L
  std::vector<void*> allocs;  // device memory owned by this level
};

// One launch of the coarse step: a level substep's sweep, or the
// coalescence that precedes it on a level with finer neighbours.
struct Op {
  enum Kind { kSweep = 0, kCoalesce = 1, kInplace = 2 };
  int level;
  int kind = kSweep;
  SweepArgs args;
  CoalArgs coal;
  InplaceArgs ia;   // kInplace: a launch of the in-place finest level
  int odd = 0;      // kInplace: 1 the odd launch (first substep), 0 the even one
};

}  // namespace lbm

struct lbm_forest {
  using LevelDev = lbm::LevelDev;
  using Forest = lbm::Forest;
  using LevelTables = lbm::LevelTables;
  Forest forest;
  std::vector<LevelTables> tabs;
  std::vector<LevelDev> lv;
  int storage = LBM_F32;
  int n = 16;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int schedule = LBM_SCHED_GRAPH;
  int persistent = 0;
  int num_cu = 256;
  bool omega_set = false;
  std::vector<int> rot;       // per level: buffer holding the current state
  std::vector<int> rot_prev;  // the same at the start of the last coarse step
  int64_t steps_since_state = 0;  // coarse steps since the state was set (init, set_pdfs, regrid)
  bool state_set = false;         // PDFs written by lbm_init_pdfs or lbm_set_pdfs
  int max_level = 0;              // deepest level a regrid may create
  double omega0 = 0.0;
  bool trt = false;               // TRT collision with a body force (lbm_set_trt_force)
  double lambda_eo = 0.0;         // Lambda_eo of eq. lambda_eo (<= 0: lambda_o = lambda_e)
  double accel0[3] = {0.0, 0.0, 0.0};  // lattice acceleration of level 0
  std::map<std::vector<int>, hipGraphExec_t> graphs;
  int* d_err = nullptr;
  bool coal_check = false;                  // FP64 accumulation check of the coalescence
  bool fuse = true;                         // forest-wide LevelDev::fuse
  bool interp = false;                      // interpolated explosion (lbm_set_explosion_interpolation)
  bool inplace = false;                     // in-place streaming (lbm_set_inplace): level 0 keeps one buffer
  int layout = 0;                           // its layout (InplaceLayout in inplace.hpp)
  bool post_lost = false;                   // in-place steps left no state of the last step's start (regrid needs it)
  int inplace_level = 0;                    // the level streamed in place (the finest; 0 on a one-level forest)
  void* save[3] = {nullptr, nullptr, nullptr};  // refined in place: saves at t (two, by parent-step parity), t + 1/2
  unsigned long long* d_check = nullptr;    // its figures (see CoalArgs::check)
  double* d_partials = nullptr;
  std::vector<void*> allocations;

  ~lbm_forest() {
    (void)hipSetDevice(device);
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    for (void* p : allocations) (void)hipFree(p);
    for (auto& v : lv)
      for (void* p : v.allocs) (void)hipFree(p);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};


namespace lbm {

// Buffer holding level L's current state: the rotating index, or buffer 0
// for the level streamed in place (whose rotation entry is then the parity
// of its parent steps).
inline int current_index(const lbm_forest* f, int L) {
  return f->inplace && L == f->inplace_level ? 0 : f->rot[L];
}
inline const void* current_state(const lbm_forest* f, int L) { return f->lv[L].buf[current_index(f, L)]; }

// Sets the thread's error message and returns `code`.
int set_error(int code, const char* fmt, ...);

// Brings the state into the natural layout (f*_a(x) at (x, a)) before a
// kernel other than the sweeps reads it: a no-op except with in-place
// streaming, whose buffer may hold the swapped or pushed layout.
int prepare_state_read(lbm_forest* f);

}  // namespace lbm
