/*
 * lbm_refined.h -- C ABI of the MI355X refined lattice Boltzmann library.
 *
 * The library advances a D3Q19 SRT lattice Boltzmann simulation on a 2:1
 * balanced forest of octrees (Schornbaum & Ruede, "Massively parallel
 * algorithms for the lattice Boltzmann method on non-uniform grids"):
 *
 *   - the domain is a grid of R_x x R_y x R_z root blocks, periodic along
 *     each axis or closed by no-slip walls (section 2.2); a block is split
 *     into 8 children of half its size; every block on every level holds
 *     n^3 cells, so level interfaces coincide with block faces
 *     (section 3.2, section 4);
 *   - neighbouring blocks differ by at most one level, counting face, edge
 *     and corner neighbours across the periodic wrap (section 2.3);
 *   - level L has grid spacing dx_0 / 2^L and time step dt_0 / 2^L
 *     (acoustic scaling) and relaxation rate
 *     omega_L = 2 omega_0 / (2^(L+1) + (1 - 2^L) omega_0)
 *     (section 2.3, eq. omega_scaling_0);
 *   - one coarse time step is NonUniformTimeStep(0) of Algorithm 1: level
 *     L+1 takes two substeps per step of level L; coarse PDFs are copied
 *     homogeneously into the fine ghost layers (explosion, eq. ctof) and the
 *     PDFs streaming from the fine ghost layers into a coarse cell are
 *     replaced by the mean of its 8 children (coalescence, eq. ftoc)
 *     (section 4, section 4.3, section 4.4).
 *
 * Conventions
 *   - Every call returns an int status: LBM_OK (0) or a negative LBM_E_*
 *     code.  No C++ exception or abort crosses the ABI.  lbm_last_error()
 *     returns a message for the calling thread's last failure.
 *   - All host arrays are owned by the caller and only read or written
 *     during the call.  All device memory is owned by the forest handle and
 *     released by lbm_destroy().
 *   - Canonical cell order: level-major (0 .. max level); inside a level,
 *     blocks sorted by the Morton (Z-order) index of their integer position
 *     on that level (x in the lowest bit); inside a block x fastest:
 *     local = i + n (j + n k).
 *   - Lattice units: rho0 = 1, c = 1 on every level.
 *   - A forest handle is used by one host thread at a time.  Device work is
 *     enqueued on the stream given at creation (the null stream if none);
 *     calls that return host data synchronize that stream.
 */
#ifndef LBM_REFINED_H
#define LBM_REFINED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define LBM_OK            0
#define LBM_E_INVALID    -1  /* null pointer, bad size, bad parameter          */
#define LBM_E_COVER      -2  /* explicit leaves do not tile the domain once     */
#define LBM_E_UNBALANCED -3  /* explicit leaves violate 2:1 and balance == 0    */
#define LBM_E_OOM        -4  /* device allocation failed                        */
#define LBM_E_HIP        -5  /* HIP runtime error (message has the HIP string)  */
#define LBM_E_NONFINITE  -6  /* a reduction found NaN or Inf                    */
#define LBM_E_STATE      -7  /* call out of order (e.g. step before omega set)  */

/* ---- storage forms ------------------------------------------------------ */
/* PDFs are stored shifted by the lattice weights, h_a = f_a - w_a, in every
 * form; arithmetic is FP64 for LBM_F64 and FP32 for the other two.          */
#define LBM_F64          0
#define LBM_F32          1
#define LBM_F16_SHIFTED  2

/* ---- schedules ------------------------------------------------------------ */
#define LBM_SCHED_GRAPH      0  /* whole coarse step captured as one hipGraph   */
#define LBM_SCHED_DIRECT     1  /* one launch per level substep, no graph        */
#define LBM_SCHED_PER_BLOCK  2  /* one launch per block per level substep: the
                                   plain "for all blocks on level L" form of
                                   Algorithm 1, kept as a comparator            */

typedef struct lbm_forest lbm_forest;

/* Refinement callback (section 3.3: user callbacks mark blocks for
 * refinement).  Asked once for every leaf of level `level` < max_level at
 * integer block position (x, y, z) of that level; nonzero = split it.  The
 * block covers [x, x + 1) x [y, y + 1) x [z, z + 1) in units of level-`level`
 * blocks, i.e. the box 2^-level (x, y, z) + [0, 2^-level)^3 in root-block
 * units; integer positions are passed instead of floating-point boxes so
 * that a callback decides exactly on the block lattice. */
typedef int (*lbm_refine_fn)(int level, int x, int y, int z, void *user);

typedef struct {
  int root_blocks[3];     /* R_x, R_y, R_z >= 1                                 */
  int cells_per_block;    /* n in {4, 8, 16, 32}                                 */
  int max_level;          /* deepest level allowed, 0 .. 20                       */
  int periodic[3];        /* per axis: 1 periodic; 0 a no-slip wall at both ends
                             (section 2.2: halfway bounce-back, the wall midway
                             between the last cell and the boundary cell beyond;
                             applied on every level and in the fine ghost
                             layers, section 4.1).  Positions beyond a wall are
                             no neighbours for the 2:1 balance.                  */
  const int32_t *leaves;  /* optional explicit leaf list [num_leaves][4] =
                             (L, x, y, z); must tile the domain exactly once    */
  int64_t num_leaves;
  lbm_refine_fn refine;   /* used when leaves == NULL: roots are split level by
                             level where refine() says so                      */
  void *refine_user;
  int balance;            /* 1: add splits until 2:1 holds (section 3.3);
                             0: an unbalanced explicit leaf list is an error.
                             Callback-built forests are always balanced.        */
  int storage;            /* LBM_F64, LBM_F32 or LBM_F16_SHIFTED                 */
  int device;             /* HIP device ordinal                                   */
  void *stream;           /* hipStream_t (e.g. torch.cuda.current_stream()
                             .cuda_stream) or NULL for the null stream         */
} lbm_forest_desc;

/* Build the balanced forest, its level tables and all device storage.
 * Errors: LBM_E_INVALID, LBM_E_COVER, LBM_E_UNBALANCED, LBM_E_OOM, LBM_E_HIP. */
int lbm_create_block_forest(const lbm_forest_desc *desc, lbm_forest **out);

/* Host only, no device work: the balanced forest that
 * lbm_create_block_forest would build from `desc`, as a canonical leaf list
 * out[count][4] = (L, x, y, z).  With out == NULL only *count is set;
 * otherwise capacity (in leaves) must be >= the count.  Same errors as
 * lbm_create_block_forest apart from device errors. */
int lbm_build_leaves(const lbm_forest_desc *desc, int32_t *out, int64_t capacity, int64_t *count);

/* Host only: lbm_level_stats of the forest `desc` describes, without
 * allocating it (sizes for planning device memory). */
int lbm_plan_level_stats(const lbm_forest_desc *desc, int level, int64_t out[8]);

/* Release all device memory and the handle.  NULL is accepted. */
int lbm_destroy(lbm_forest *f);

/* Levels, blocks and interior cells.  level == -1 sums over all levels. */
int lbm_num_levels(const lbm_forest *f, int *num_levels);
int lbm_num_blocks(const lbm_forest *f, int level, int64_t *num_blocks);
int lbm_num_cells(const lbm_forest *f, int level, int64_t *num_cells);

/* Leaves in canonical order, out[num_blocks(-1)][4] = (L, x, y, z). */
int lbm_get_leaves(const lbm_forest *f, int32_t *out);

/* Per-level layout figures, out[8] = { blocks, blocks touching level L-1,
 * interior cells, blocks touching level L+1, work tiles of the sweep,
 * coalesced (cell, direction) pairs, bytes per stored PDF, cells per block }. */
int lbm_level_stats(const lbm_forest *f, int level, int64_t out[8]);

/* Relaxation rates omega_L of all levels from omega_0 by eq. omega_scaling_0
 * (section 2.3).  0 <= omega0 < 2; omega0 == 0 switches collision off
 * (pure advection, a test mode).  Must be called before lbm_step_coarse. */
int lbm_set_level_omega(lbm_forest *f, double omega0);
int lbm_get_level_omega(const lbm_forest *f, int level, double *omega);

/* TRT collision and a constant body force (section 2, TRT model and
 * external forces).  omega_L of lbm_set_level_omega becomes the even rate
 * lambda_e,L; lambda_eo > 0 is Lambda_eo of eq. lambda_eo, kept on every
 * level by lambda_o,L from eq. lambda_oL (lambda_eo == 0: lambda_o = lambda_e).
 * accel0[3] (host, may be NULL for none) is the lattice acceleration a_0* of
 * level 0; level L uses a_0* / 2^L (eq. force_scaling) and adds
 * F_a = 3 w_a e_a . a_L after each collision, with u in f^eq the plain sum
 * e f.  lambda_eo == 0 with no acceleration restores SRT.  The acceleration
 * is set before lbm_init_pdfs: the stored state is post-collision, and
 * lbm_init_pdfs (and lbm_set_pdfs, whose input is taken as such a state)
 * includes the force term of one collision; once PDFs are set, a call with a
 * different acceleration returns LBM_E_STATE (lambda_eo alone may change).
 * lbm_get_moments then reports u = sum e f / rho0 + a_L / 2 of the
 * pre-collision state, and lbm_mass the momentum of the stored
 * (post-collision) state, which holds a_L / 2 more per unit mass than the
 * pre-collision one.  lbm_regrid refuses a forest with TRT or a force
 * (LBM_E_STATE).
 * Errors: LBM_E_INVALID (null handle, lambda_eo < 0 or not finite, a
 * non-finite acceleration), LBM_E_STATE (acceleration changed after the
 * PDFs were set). */
int lbm_set_trt_force(lbm_forest *f, double lambda_eo, const double accel0[3]);

/* f = f^eq(rho, u) (eq. fequ) on every interior cell.  rho[N], u[N][3],
 * host FP64 in canonical order, N = lbm_num_cells(-1).  Synchronous. */
int lbm_init_pdfs(lbm_forest *f, const double *rho, const double *u);

/* Advance n_steps >= 0 coarse time steps (Algorithm 1 from level 0), with
 * the schedule set by lbm_set_schedule.  Asynchronous on the stream. */
int lbm_step_coarse(lbm_forest *f, int n_steps);

/* Density and velocity of every interior cell (eq. fvelocity read as
 * rho = sum f, u = sum e f / rho0), host FP64 in canonical order.  With a
 * body force (lbm_set_trt_force) the stored post-collision state carries the
 * force term F_a = 3 w_a e_a . a_L, and u = sum e f / rho0 - a_L / 2 of it,
 * which is the paper's velocity sum e f / rho0 + a_L / 2 of the
 * pre-collision state (section 2, external forces).
 * Synchronizes the stream. */
int lbm_get_moments(lbm_forest *f, double *rho, double *u);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * output as lbm_get_moments, computed by the same kernel, without any
 * allocation.  The cells pass through a staging array of the library's own
 * that each device holds for the life of the process (16 MiB: chunks of at
 * most 524,288 cells, so any forest size is accepted).  Every call on a
 * device shares that device's array: calls that overlap on one device (from
 * several threads, or forests on different streams) race and must be
 * serialized by the caller.  Synchronizes the forest's stream.
 * Errors: LBM_E_INVALID, LBM_E_STATE (a failed table lookup in an earlier
 * sweep), LBM_E_HIP. */
int lbm_get_moments_static(lbm_forest *f, double *rho, double *u);

/* Volume-weighted mass and momentum, M = sum_L 8^-L sum_{cells} sum_a f_a
 * and J = sum_L 8^-L sum sum e_a f_a, accumulated in FP64 on the device.
 * The weight of a level-L cell is its volume (dx_L / dx_0)^3 = 8^-L in
 * units of a level-0 cell, as in the volume-weighted error norms of the
 * validation (section 5.1); the volume-based scheme conserves M across
 * levels (section 4.4).  The sum covers the stored (post-collision) state.
 * LBM_E_NONFINITE if NaN or Inf appears.  Synchronizes the stream. */
int lbm_mass(lbm_forest *f, double *mass, double momentum[3]);

/* Interpolated explosion (on != 0; off by default: the homogeneous
 * explosion of eq. ctof).  Algorithm 2 refines the homogeneous explosion by
 * an interpolation of the exploded values (section 4.1) whose scheme the
 * paper only cites; the library's reading: every PDF of a fine ghost cell is
 * reconstructed linearly inside its coarse parent P, f_a(P) + sum_d
 * (o_d - 1/2)/2 g_d with o the cell's octant in P and g_d the minmod-limited
 * slope from P's two face neighbours along axis d (0 where either is not an
 * interior cell of P's level, a wall included).  The 8 children of a parent
 * average to its values, so mass and momentum are kept, and zero slopes give
 * eq. ctof.  It applies to every exploded value the sweeps and the
 * coalescence read; lbm_regrid still explodes whole new blocks
 * homogeneously.  Invalidates captured graphs.  LBM_E_STATE for on != 0
 * while a refined forest streams in place. */
int lbm_set_explosion_interpolation(lbm_forest *f, int on);

/* In-place streaming (on != 0; off by default).  Section 4.1 stores two
 * grids, source and destination, and names the AA pattern as the in-place
 * alternative that refinement does not readily admit.  The library streams
 * the finest level in place: it keeps one PDF buffer instead of two (a
 * forest of one level) or three (the finest level of a refined forest);
 * the bytes moved per cell update stay 38 s (19 values read and 19
 * written).  The finest level's steps alternate an odd launch (pull from
 * the neighbours, collide, push to them) and an even one (collide in
 * place); on a refined forest they are its first and second substeps, the
 * explosion reads the parent level's current state, and the values the
 * finest cells send into the fine ghost layers (section 4) at t and t + 1/2
 * are saved for the second substep's back-trace and the coarser level's
 * coalescence (30 n^2 values per block, three arrays).  The buffer holds the
 * post-collision state in a layout that alternates with the launches and is
 * brought back to the natural layout, in place, before lbm_get_moments,
 * lbm_get_moments_static, lbm_mass, lbm_get_pdfs or the indicator calls
 * read it.  Results equal those of two-buffer streaming bitwise, SRT and
 * TRT with a body force, periodic axes and no-slip walls alike.  on = 1
 * frees the finest level's other buffers (after synchronizing the stream;
 * one x-face buffer stays, to hold the values that cross x faces); on = 0
 * allocates them again.  While on, lbm_autotune and lbm_regrid return
 * LBM_E_STATE, and lbm_regrid also does until a coarse step with
 * two-buffer streaming has been taken (it needs the state at the start of
 * the last coarse step).  Invalidates captured graphs.  Errors:
 * LBM_E_INVALID (on not 0 or 1), LBM_E_STATE (on = 1 on a refined forest
 * with the interpolated explosion, which then stays off), LBM_E_OOM,
 * LBM_E_HIP. */
int lbm_set_inplace(lbm_forest *f, int on);

/* Whether in-place streaming is on (*on = 1) or off (0). */
int lbm_get_inplace(const lbm_forest *f, int *on);

/* Free and total device memory of `device` in bytes (hipMemGetInfo): for
 * sizing forests, and to see the memory lbm_set_inplace releases.  Errors:
 * LBM_E_INVALID, LBM_E_HIP. */
int lbm_device_memory(int device, int64_t *free_bytes, int64_t *total_bytes);

/* FP64 accumulation check of the coalescence (eq. ftoc, section 4.4).  With
 * FP32 or FP16 storage the 8-child sums are formed in FP32; with the check
 * on (on != 0; off by default) every coalescence launch also sums the same
 * loaded values in FP64.  The stored results do not change.  Invalidates
 * captured graphs. */
int lbm_set_coalescence_check(lbm_forest *f, int on);

/* Figures of the check since the last call, which resets them:
 * out[0] = largest |mean - FP64 mean| over the coalesced pairs, out[1] =
 * largest ratio |sum - FP64 sum| / (gamma_7 sum |v|), gamma_7 = 7u/(1 - 7u)
 * the error bound of recursive summation of 8 terms in the compute type of
 * unit roundoff u (at most 1 for a correct sum), out[2] = pairs checked.
 * Synchronizes the stream. */
int lbm_coalescence_check(lbm_forest *f, double out[3]);

/* Where the coalescence of level L (eq. ftoc) runs (Algorithm 1 places it
 * after level L+1's two substeps and before level L's next stream).  With
 * fusion on for level L+1: inside the launch of level L+1's second substep,
 * whose workgroups it shares, when that launch has one workgroup per work
 * tile and the homogeneous explosion; its inputs (level L+1's states at t
 * and t + 1/2, level L's current state) are ones that substep does not
 * write.  Otherwise, and on the per-block schedule, with a persistent grid
 * on level L+1, the interpolated explosion or an in-place level L+1: a launch
 * of its own before level L's sweep.  Results are bitwise the same either
 * way.  lbm_set_coalescence_fusion sets every level (on = 1, the default, or
 * 0; also for levels a regrid creates); lbm_set_level_fusion sets one level
 * (on = 1, 0, or -1 for the forest-wide setting; kept across lbm_regrid for
 * levels that still exist), and the autotuner picks it per level;
 * lbm_get_level_fusion gives the setting in force (1 or 0).  Invalidate
 * captured graphs.  Errors: LBM_E_INVALID (null pointer, level out of range,
 * on out of range). */
int lbm_set_coalescence_fusion(lbm_forest *f, int on);
int lbm_set_level_fusion(lbm_forest *f, int level, int on);
int lbm_get_level_fusion(const lbm_forest *f, int level, int *on);

/* Schedule of lbm_step_coarse: LBM_SCHED_GRAPH (default), _DIRECT or
 * _PER_BLOCK.  All three give bitwise identical results. */
int lbm_set_schedule(lbm_forest *f, int schedule);

/* Launch shape of the sweep kernel: persistent > 0 runs `persistent`
 * workgroups per compute unit that loop over the level's work tiles;
 * persistent == 0 launches one workgroup per tile.  Invalidates a captured
 * graph.  Results do not depend on it. */
int lbm_set_launch(lbm_forest *f, int persistent);

/* Launch shape of one level's sweep: persistent as in lbm_set_launch (-1:
 * follow the forest-wide setting); order 0 sweeps the work tiles in
 * canonical order, order 1 maps workgroups to work units so that each of
 * the 8 XCDs (to which workgroups are dispatched round-robin) sweeps one
 * contiguous range of them; split (1, 2 or 4) sweeps each work tile with
 * that many workgroups
 * of 256 / split lanes (the largest allowed split <= the request is used:
 * a workgroup keeps at least one full wavefront).  Synchronizes the stream;
 * invalidates captured graphs; kept across lbm_regrid for levels that still
 * exist.  Results do not depend on it. */
int lbm_set_level_launch(lbm_forest *f, int level, int persistent, int order, int split);
int lbm_get_level_launch(const lbm_forest *f, int level, int *persistent, int *order, int *split);

/* Autotuner of the launch shape (the batching form: every level's tiles in
 * one launch per substep, the step captured as a graph).  Times each
 * candidate (persistent, order, split) -- one workgroup per work unit with
 * order {0, 1} x split {1, 2, 4}, and persistent grids of {1, 2, 4, 8}
 * workgroups per CU with order {0, 1} -- each with the coarser level's
 * coalescence fused into the level's second substep and in a launch of its
 * own (lbm_set_level_fusion), with lbm_time_launches over one warm-up and
 * n_steps >= 1 coarse steps, in two passes over all candidates (each
 * candidate keeps its faster pass), keeps for every level the candidate
 * with the smallest mean step time of that level (its two substeps plus the
 * coarser level's coalescence launch where that runs on its own), and
 * applies it.  With TRT (lbm_set_trt_force) a persistent candidate runs one
 * workgroup per work unit.
 * result[5 * L + {0, 1, 2, 3, 4}] = chosen persistent, order, split, fusion
 * and that level's mean time per level step in ms.  The PDF state is saved before
 * and restored after (device memory equal to the forest's PDF storage is
 * allocated for it; LBM_E_OOM otherwise), so the simulation is left exactly
 * where it was.  Synchronizes. */
int lbm_autotune(lbm_forest *f, int n_steps, double *result);

/* Dynamic regrid (the paper names dynamic refinement as future work; the
 * operators are its own).  flags[i] for the i-th leaf in canonical order:
 * > 0 split it (if below the max_level given at creation), < 0 merge it with
 * its 7 siblings if all 8 are leaves flagged < 0, 0 keep.  Order: splits,
 * 2:1 balance by further splits, then merges from the finest level down,
 * each kept only if no leaf two levels finer than the merged parent touches
 * it.  PDFs: unchanged blocks keep their state; a new fine block takes, in
 * all 19 directions, the post-streaming values of the coarse cell containing
 * each cell (eq. ctof), a merged block the mean of its 8 children (eq. ftoc),
 * and is then collided.  count = number of leaves.  Synchronous; afterwards
 * sizes, leaves and the canonical order refer to the new forest. */
int lbm_regrid(lbm_forest *f, const int8_t *flags, int64_t count);

/* Instrumented stepping: advance n_steps >= 1 coarse steps with direct
 * launches, a hipEvent pair on the forest's stream around every sweep, and
 * return the mean launch duration in milliseconds and the launch count per
 * (level, substep): ms[L * 2 + s - 1], launches[L * 2 + s - 1] for
 * L < num_levels, s in {1, 2} (level 0 only has s = 1).  Synchronizes. */
int lbm_time_sweeps(lbm_forest *f, int n_steps, double *ms, int64_t *launches);

/* The same, also timing the coalescence launches (one before each sweep of
 * a level with finer neighbours): coal_ms[L], coal_launches[L] for
 * L < num_levels (0 where there is none).  coal_ms and coal_launches are
 * both given or both NULL. */
int lbm_time_launches(lbm_forest *f, int n_steps, double *ms, int64_t *launches, double *coal_ms,
                      int64_t *coal_launches);

/* Wait for all work enqueued by this forest. */
int lbm_synchronize(lbm_forest *f);

/* Raw shifted PDFs h = f - w of every interior cell, FP64, canonical order,
 * layout [cell][19] with the direction order of lbm_lattice().  For exact
 * checkpoint/resume (moments alone lose the non-equilibrium part). */
int lbm_get_pdfs(lbm_forest *f, double *h);
int lbm_set_pdfs(lbm_forest *f, const double *h);

/* The D3Q19 velocity set used for raw PDF I/O: e[19][3], w[19]. */
int lbm_lattice(int32_t *e, double *w);

/* ---- refinement indicators and the learned surrogate ------------------------
 * The paper leaves the refinement criterion to the user (section 3.3); the
 * definitions below are this library's.  Per block, on the stored
 * (post-collision) state: I_omega = max over cells of |curl u| with
 * block-local differences in the block's lattice units; I_neq = mean over
 * cells of ||f - f_eq|| / rho.  A block is refine-worthy if I_omega >
 * theta_omega or I_neq > theta_neq, coarsen-worthy if both are below half
 * their threshold, kept otherwise. */

/* Per block in canonical order: features[nblocks][12] = { level / Lmax,
 * 1e3 mean(rho - 1), log10(x + 1e-12) of: std rho, |mean u|,
 * rms |u - mean u|, max |u|, octant-mean jumps of u along x, y, z, |curl| of
 * the 2x2x2 octant-mean field, mean neq, max neq } and
 * crit[nblocks][2] = { I_omega, I_neq }.  Host FP64 outputs; synchronizes. */
int lbm_block_indicators(lbm_forest *f, double *features, double *crit);

/* The same features[nblocks][12] from one fused pass over the PDFs (no
 * per-cell intermediates, no curl stencil): the MLP's input path. */
int lbm_block_features(lbm_forest *f, double *features);

/* Soft targets of the criterion for given crit[n][2]: 1 refine-worthy,
 * 0 coarsen-worthy, 0.5 keep (host computation). */
int lbm_plain_targets(const double *crit, int64_t n, double theta_omega, double theta_neq, double *target);

/* MLP 12 -> 64 -> 64 -> 1 (ReLU, sigmoid), FP32 on the device, trained with
 * the library's own forward, backward and Adam kernels on the mean binary
 * cross entropy against soft targets (1 refine, 0.5 keep, 0 coarsen).
 * Parameters packed W1[64][12], b1[64], W2[64][64], b2[64], w3[64], b3
 * (5057 floats).  Inputs are normalized as (x - mean) / std. */
typedef struct lbm_mlp lbm_mlp;
int lbm_mlp_create(int device, uint64_t seed, lbm_mlp **out);   /* He init from seed */
int lbm_mlp_destroy(lbm_mlp *m);
int lbm_mlp_num_params(int *n);
int lbm_mlp_get_params(lbm_mlp *m, float *params);
int lbm_mlp_set_params(lbm_mlp *m, const float *params);        /* resets Adam state */
/* mean, std: [12]; fmin, fmax: [12] training range (NULL = unbounded); a
 * feature outside it sends the decision to the criterion. */
int lbm_mlp_set_normalization(lbm_mlp *m, const double *mean, const double *std, const double *fmin,
                              const double *fmax);
/* mean, std (floor 1e-6), min and max of the features X[n][12]. */
int lbm_mlp_fit_normalization(lbm_mlp *m, const double *X, int64_t n);
int lbm_mlp_predict(lbm_mlp *m, const double *X, int64_t n, float *prob);        /* X[n][12] */
int lbm_mlp_gradient(lbm_mlp *m, const double *X, const double *target, int64_t n, float *grad);
/* Adam (beta 0.9, 0.999), shuffled minibatches of `batch` samples (a
 * trailing partial batch is skipped), epoch_loss[epochs] (may be NULL). */
int lbm_mlp_train(lbm_mlp *m, const double *X, const double *target, int64_t n, int epochs, int batch, double lr,
                  uint64_t seed, double *epoch_loss);

/* Regrid flags (for lbm_regrid) per block in canonical order: +1 refine,
 * -1 coarsen, 0 keep (refine only below max_level, coarsen only above
 * level 0).  With m == NULL the criterion decides (two passes over the
 * cells: moments, then the curl stencil); otherwise the features come from a
 * single fused pass, the MLP decides (p > 0.75 refine, p < 0.25 coarsen),
 * and the criterion is evaluated only for blocks where p lies within delta
 * of 0.25 or 0.75 or a feature is outside the training range;
 * *n_fallback (may be NULL) counts those blocks. */
int lbm_refinement_flags(lbm_forest *f, lbm_mlp *m, double theta_omega, double theta_neq, double delta,
                         int8_t *flags, int32_t *n_fallback);

/* Message of the calling thread's last error ("" if none). */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_REFINED_H */
