// Kernel launch interface shared by the API layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

// Coalescence of level L for one of its substeps (eq. ftoc), run after the
// finer level's two substeps and before the level-L sweep: for every
// coalesced pair (X, a) of a slot with finer neighbours, the mean over the 8
// children of X of what the finer level's second stream pulled into them
// (with the bounce-back at no-slip walls in the fine ghost layers),
// written to out[row][a][cell] (block-major like the state, one block per
// fine_nbr row), or to out_x for a pair that enters through an x face
// (cell x = 0 with e_a,x = +1, x = n - 1 with e_a,x = -1; x-face layout).
//
// Every state buffer has an x-face copy, [slot][10][n^2]: the values that
// leave each block through its x faces (cell x = 0 for e_a,x = -1, x = n - 1
// for +1).  Each sweep writes the copy of the buffer it writes, from
// registers.  The sweep takes the x-edge value of each row end from its x
// neighbour's copy, and the coalescence its children at x faces; in the
// state's layout each of these would cost a 128-byte line per element.  A
// buffer written by anything but a sweep has its copy refreshed by
// launch_face_copy.
struct CoalArgs {
  const void* cur;            // level-L state read by the following sweep (the regular sources)
  const void* fine0;          // level-(L+1) state at the start of the parent step
  const void* fine1;          // level-(L+1) state after its first substep
  void* out;                  // [row][19][n^3]
  void* out_x;                // [row][10][n^2]
  const void* fine0_x;        // x-face copies of fine0 and fine1
  const void* fine1_x;
  const uint16_t* cells;      // [pair]: the pair's cell, grouped by row, then direction
  const int32_t* chunks;      // [chunk][4]: fine_nbr row, coarse slot, first pair, count |
                              // (direction << 16); count 0: nothing to do
  int32_t nchunks;
  const int32_t* nbr;         // level-L [slot][27]
  const int32_t* fine_nbr;    // [row][8][27]
  const int32_t* fine_slot;   // [row]
  // accumulation check (null: off): each pair's 8-child sum is also formed
  // in FP64 from the same loaded values; check[0] and check[1] keep, as the
  // bit patterns of non-negative doubles, the largest |compute-type mean -
  // FP64 mean| and the largest ratio of |sum - FP64 sum| to the bound
  // gamma_7 sum |v| of recursive summation of 8 terms; check[2] counts pairs
  unsigned long long* check;
  int* err;                   // error bits (table lookup failures)
  int32_t interp;             // 1: interpolated explosion of the coarse values the children trace back to
  int32_t walls;              // 1: the forest has a non-periodic axis (no-slip walls)
  // finer level streamed in place (non-null): its values at t and t + 1/2 come
  // from its save arrays instead of fine0 / fine1 (see inplace_save.hpp)
  const void* save_t;         // saves of the finer state at the start of its parent step
  const void* save_half;      // saves of the finer state after its first substep
};

// Arguments of one level substep of the fused sweep.  PDF buffers are
// block-major: element (a, slot, cell) sits at (19 slot + a) n^3 + cell.
// Levels L >= 1 keep three buffers: the state at the start of the parent
// step (t), after the first substep (t + 1/2) and after the second (t + 1).
struct SweepArgs {
  const void* cur;            // level-L state read by this substep (t or t + 1/2)
  const void* prev;           // level-L state at t (second substep only)
  void* nxt;                  // level-L state written
  const void* par;            // level-(L-1) post-collision state (explosion source)
  const void* par_face;       // its x-face copy (parent values at the parent's x faces)
  const void* fine0;          // level-(L+1) state at the start of its last parent step
  const void* fine1;          // level-(L+1) state after the first of its two substeps
  const int32_t* work;        // work tiles (slot * tiles_per_block + tile), or null: tiles work0 + [0, nwork)
  int32_t work0;
  int32_t nwork;
  int32_t xcd;                // 1: work units grouped by XCD (see xcd_unit in the sweep)
  int32_t substep;            // 1 or 2
  int32_t collide;            // 1: collide interior cells (normal); 0: write the streamed values
  const int32_t* nbr;         // [slot][27]
  const uint32_t* flags;      // [slot]
  const int32_t* fine_index;  // [slot]
  const void* coal;           // coalesced values of this substep, [row][19][n^3] (see CoalArgs)
  const void* coal_x;         // the same for the pairs entering through an x face, [row][10][n^2]
  const void* face_cur;       // x-face copy of cur, [slot][10][n^2] (see CoalArgs)
  void* face_out;             // x-face copy of nxt (null: not written)
  float omega;                // omega_L (FP32 arithmetic forms); lambda_e,L with trt
  double omega64;             // omega_L (FP64 form)
  int* err;                   // error bits (table lookup failures)
  int32_t trt;                // 1: TRT collision with a body force (the fields below)
  float lambda_o;             // lambda_o,L (FP32 arithmetic forms)
  double lambda_o64;          // lambda_o,L (FP64 form)
  float accel[3];             // lattice acceleration a_L (FP32 arithmetic forms)
  double accel64[3];          // a_L (FP64 form)
  int32_t interp;             // 1: interpolated explosion (see interp_value in lattice.hpp)
  const int32_t* par_nbr;     // level-(L-1) [slot][27] (the parents' neighbours, for interp)
  // the coalescence of level L - 1 run by this launch (a second substep of
  // level L with one workgroup per work unit and the homogeneous explosion):
  // fc.nchunks workgroups, one per chunk, interleaved with the sweep's work
  // units (launch_sweep sets the spacing); fc.nchunks = 0: none.  The chunks
  // read only level L's states at t and t + 1/2 and level L - 1's current
  // state, none of which this substep writes.
  CoalArgs fc;
  int32_t fc_stride;
};

enum ErrBits : int { kErrNoSource = 1, kErrNoChild = 2 };

hipError_t launch_coalesce(int storage, int n, const CoalArgs& a, hipStream_t stream);

// x-face copy of a whole buffer of nblocks blocks.
hipError_t launch_face_copy(int storage, int n, const void* buf, void* xf, int64_t nblocks, hipStream_t stream);

// Cells per work tile of the sweep kernel (one workgroup's share).
int sweep_tile_cells(int storage, int n);

// Workgroup split of the sweep: each work tile is swept by `split` (1, 2
// or 4) workgroups of 1 / split of the lanes.  sweep_split returns the
// largest split <= requested that keeps a full wavefront per workgroup.
int sweep_split(int storage, int n, int requested);

// storage: 0 = f64, 1 = f32, 2 = f16.  grid >= nwork * split launches one
// workgroup per work unit; a smaller grid is persistent.
hipError_t launch_sweep(int storage, int n, const SweepArgs& a, int grid, int split, hipStream_t stream);

// The helpers below address the interior cells [0, ncells) of one level
// (block-major buffer: element (a, slot, cell) at (19 slot + a) n^3 + cell).

// Lattice acceleration of one level (zero: no body force).
struct Accel {
  double a[3];
};

// h = f^eq(rho, u) - w, plus the force term F_a = 3 w_a e_a . a of a
// collision: the stored state is post-collision, and collision leaves an
// equilibrium unchanged apart from the force.
hipError_t launch_init(int storage, int n, void* buf, const double* rho, const double* u,
                       int64_t ncells, Accel accel, hipStream_t stream);

// rho = 1 + sum h, u = sum e h - a / 2: the velocity of the pre-collision
// state (sum e h - a) plus a / 2 (section 2, external forces).  Cells
// [first, first + count) of the level; rho[count], u[count][3].
hipError_t launch_moments(int storage, int n, const void* buf, double* rho, double* u, int64_t first,
                          int64_t count, Accel accel, hipStream_t stream);

// Raw shifted PDFs, FP64 [cell][19].
hipError_t launch_get_pdfs(int storage, int n, const void* buf, double* h, int64_t ncells,
                           hipStream_t stream);
hipError_t launch_set_pdfs(int storage, int n, void* buf, const double* h, int64_t ncells,
                           hipStream_t stream);

// FP64 partial sums (sum h, sum e_x h, sum e_y h, sum e_z h, nonfinite count);
// kReduceGrid workgroups write out[kReduceGrid][5].
constexpr int kReduceGrid = 1024;
hipError_t launch_reduce(int storage, int n, const void* buf, int64_t ncells, double* out,
                         hipStream_t stream);

// Regrid remap of one new level.  Each new block takes its PDFs from the old
// forest: mode 0 copies an unchanged block from the old state; mode 1
// explodes an old ancestor `shift` levels up (eq. ctof: a new cell takes the
// cell containing it, local offset `off` inside the old block); mode 2
// averages the 8 old child blocks (eq. ftoc).  Modes 1 and 2 read the old
// post-streaming values and collide the result with omega when collide != 0.
struct RemapBlock {
  int32_t mode;
  int32_t src_level;
  int32_t shift;
  int32_t off[3];
  int32_t slot[8];
};

struct RemapArgs {
  void* dst;                  // new level buffer
  const RemapBlock* blocks;   // one per new block
  int64_t ncells;             // new blocks * n^3
  const void* const* old_cur;   // per old level: current (post-collision) state
  const void* const* old_post;  // per old level: post-streaming values of changed blocks
  int32_t collide;
  float omega;
  double omega64;
};

hipError_t launch_remap(int storage, int n, const RemapArgs& a, hipStream_t stream);

}  // namespace lbm
