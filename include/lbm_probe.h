/*
 * lbm_probe.h -- bandwidth probes of the MI355X refined lattice Boltzmann
 * library (measurement helpers, not part of the time step).
 *
 * They give the ceilings that the sweep's achieved HBM bandwidth is read
 * against: a plain device copy, and a kernel with the sweep's own memory
 * access shape (per work tile, 19 direction rows of one block read and 19
 * written, the block-major layout [block][19][n^3] of the PDF buffers) and
 * no arithmetic.  The fused stream-collide update of section 4 moves 19
 * PDFs in and 19 out per cell, so this is the traffic a sweep at the memory
 * bound cannot beat.
 *
 * Conventions as in lbm_refined.h: int status (LBM_OK or a negative
 * LBM_E_* code), lbm_last_error() for the message.  The caller owns all
 * buffers (device pointers, e.g. from torch tensors); the probes allocate
 * nothing.  Work is enqueued on `stream` (hipStream_t, NULL = null stream)
 * and timed with a pair of HIP events on that stream; every call
 * synchronizes the stream before it returns.
 */
#ifndef LBM_PROBE_H
#define LBM_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Copy `bytes` (a multiple of 16, > 0) from src to dst (16-byte aligned,
 * not overlapping) with 16-byte loads and stores, `iters` >= 1 times;
 * nontemporal != 0 stores past the caches as the sweep does.  ms = mean
 * time of one copy in milliseconds.  Errors: LBM_E_INVALID, LBM_E_HIP. */
int lbm_probe_copy(void *dst, const void *src, int64_t bytes, int iters, int nontemporal, void *stream,
                   double *ms);

/* The sweep's access shape without arithmetic: src and dst hold nblocks
 * blocks of 19 rows of n^3 elements of `elem_bytes` (2, 4 or 8) each,
 * n = cells_per_block in {16, 32}.  Every workgroup of `lanes` (64, 128 or
 * 256) threads takes lanes * 16 / elem_bytes consecutive cells of one
 * block, loads its 19 rows (16 bytes per lane and row, all loads in flight
 * before the first store) and stores them to dst.  xcd != 0 maps
 * workgroups so that each of the 8 XCDs sweeps one contiguous range of
 * tiles, as the sweep's XCD-grouped order.  `iters` >= 1 launches; ms =
 * mean launch time.  Errors: LBM_E_INVALID, LBM_E_HIP. */
int lbm_probe_streams(void *dst, const void *src, int64_t nblocks, int cells_per_block, int elem_bytes, int lanes,
                      int xcd, int iters, void *stream, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* LBM_PROBE_H */
