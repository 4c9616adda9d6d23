// In-place streaming (the AA pattern) for forests whose blocks all lie on
// one level: one PDF buffer instead of two.
//
// Section 4.1 uses two grids (source and destination) and names the AA
// pattern as the in-place alternative that refinement does not readily
// admit.  Here it is built for forests without level interfaces.  The
// buffer always holds the post-collision state f* of the last step, in one
// of three layouts:
//   natural: f*_a(x) at (x, a), the layout of the two-buffer path;
//   swapped: f*_a(x) at (x, opp(a));
//   pushed:  f*_a(x) at (x + e_a, a), the pre-collision value of the next
//            step, or at (x, opp(a)) where x + e_a lies beyond a wall
//            (halfway bounce-back, section 2.2); a value whose place is a
//            cell at an x face that it enters through (x = 0 for
//            e_a,x = +1, x = n - 1 for e_a,x = -1) is held in the entry
//            buffer (x-face layout) instead.
// The odd launch takes swapped to pushed: cell x reads f*_a(x - e_a) at
// (x - e_a, opp(a)) (its own (x, a) where x - e_a is a wall), collides and
// writes f*_a(x) to (x + e_a, a).  The even launch takes pushed to swapped:
// cell x reads (x, a), collides and writes (x, opp(a)).  In both, every
// memory location is read and then written by the one cell that owns it, so
// the buffer is updated in place without races.  Both launches do the
// two-buffer sweep's arithmetic on the same values, so results are bitwise
// those of the two-buffer path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

enum InplaceLayout : int { kLayoutNatural = 0, kLayoutSwapped = 1, kLayoutPushed = 2 };

// Arrays of n^2 values per block in each save array of a refined forest's
// in-place level (inplace_save.hpp).
constexpr int kSaveArrayCount = 30;

struct InplaceArgs {
  void* buf;             // the level's PDF buffer, block-major [slot][19][n^3]
  void* face;            // x-face copy [slot][10][n^2]: written by the even launch, read by the odd one
  void* entry;           // entry buffer [slot][10][n^2]: written by the odd launch, read by the even one
  const int32_t* nbr;    // [slot][27]: slot or kNbrWall
  int32_t nblocks;
  int32_t xcd;           // 1: work units grouped by XCD
  int32_t trt;           // 1: TRT collision with a body force
  float omega;           // omega (SRT) or lambda_e (TRT), FP32 arithmetic forms
  float lambda_o;
  float accel[3];
  // the finest level of a refined forest (refined != 0; see inplace_save.hpp)
  int32_t refined;
  const uint32_t* flags; // [slot] SlotFlags
  const void* par;       // level-(L-1) current state (two buffers): explosion source
  const void* par_face;  // its x-face copy (parents on the parent block's x faces)
  const void* save_in;   // saves of the state at the start of the parent step (second substep reads)
  void* save_out;        // saves written: t + 1/2 (first substep), t + 1 (second substep)
  int* err;              // error bits (table lookup failures)
  double omega64;        // the same for the FP64 form
  double lambda_o64;
  double accel64[3];
};

// Workgroups of one launch (each sweeps a tile of one block).
int64_t inplace_grid(int storage, int n, int64_t nblocks);

// odd = true: swapped -> pushed; false: pushed -> swapped.
hipError_t launch_inplace(int storage, int n, const InplaceArgs& a, bool odd, hipStream_t stream);

// natural <-> swapped: per cell, (x, a) <-> (x, opp(a)).
hipError_t launch_inplace_swap(int storage, int n, void* buf, int64_t nblocks, hipStream_t stream);

// Saves of the finest level's state (natural layout) at the start of a
// parent step (inplace_save.hpp).
hipError_t launch_inplace_save_fill(int storage, int n, const void* buf, void* save, const int32_t* nbr, int64_t nblocks,
                                    hipStream_t stream);

// Pushed layout: the entry buffer's values back into the buffer (before
// launch_inplace_pair_swap converts it).
hipError_t launch_inplace_entry_merge(int storage, int n, void* buf, const void* entry, int64_t nblocks,
                                      hipStream_t stream);

// pushed <-> swapped: (x, a) <-> (x - e_a, opp(a)) for every cell x and
// direction a whose neighbour x - e_a is a cell (walls: fixed points).
hipError_t launch_inplace_pair_swap(int storage, int n, void* buf, const int32_t* nbr, int64_t nblocks,
                                    hipStream_t stream);

}  // namespace lbm
