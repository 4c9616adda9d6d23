// Kernel launch interface shared by the API layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

// Arguments of one level substep of the fused sweep.
struct SweepArgs {
  const void* cur;            // level-L PDFs read by this substep  [slot][19][n^3]
  void* nxt;                  // level-L PDFs written               [slot][19][n^3]
  const void* par;            // level-(L-1) PDFs (post-collision) for the explosion gather
  const void* fine;           // level-(L+1) PDFs after its two substeps, for coalescence
  const int32_t* work;        // work tiles: slot * tiles_per_block + tile
  int32_t nwork;
  int32_t nreal;              // slots [0, nreal) are real blocks
  const int32_t* nbr;         // [slot][27]
  const uint32_t* zmask;      // [slot]
  const int32_t* parent;      // [slot]
  const int32_t* child_ghost; // [real slot][8]
  const uint32_t* flags;      // [slot]
  int32_t substep;            // 1: all non-interior sources come from the parent
                              // 2: halo sources come from the level's own halo
  float omega;                // omega_L (FP32 arithmetic forms)
  double omega64;             // omega_L (FP64 form)
  int* err;                   // error bits (table lookup failures)
};

enum ErrBits : int { kErrNoSource = 1, kErrNoChild = 2 };

// storage: 0 = f64, 1 = f32, 2 = f16
hipError_t launch_sweep(int storage, int n, const SweepArgs& a, int grid, hipStream_t stream);

// h = f^eq(rho, u) - w on the interior cells [0, ncells) of one level.
hipError_t launch_init(int storage, int n, void* buf, const double* rho, const double* u, int64_t ncells,
                       hipStream_t stream);

// rho = 1 + sum h, u = sum e h on the interior cells of one level.
hipError_t launch_moments(int storage, int n, const void* buf, double* rho, double* u, int64_t ncells,
                          hipStream_t stream);

// Raw shifted PDFs of the interior cells, FP64 [cell][19].
hipError_t launch_get_pdfs(int storage, int n, const void* buf, double* h, int64_t ncells, hipStream_t stream);
hipError_t launch_set_pdfs(int storage, int n, void* buf, const double* h, int64_t ncells, hipStream_t stream);

// FP64 partial sums (sum h, sum e_x h, sum e_y h, sum e_z h, nonfinite count)
// of the interior cells; `grid` workgroups write out[grid][5].
constexpr int kReduceGrid = 1024;
hipError_t launch_reduce(int storage, int n, const void* buf, int64_t ncells, double* out, hipStream_t stream);

}  // namespace lbm
