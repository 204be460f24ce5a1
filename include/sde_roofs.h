/* Measured ceilings of the operations the transport kernel is built from.
 *
 * The transport step (the Euler-Maruyama step of Eq. (VSDE) with the jump
 * clock of Eq. (Npi) and the voxel tally) is priced in VALU issue slots, with
 * transcendentals and 32x32->64 products weighted as quarter-rate, and its
 * tally in int64 atomics.  These entry points time each ingredient alone on
 * the current device so that those weights and ceilings are measured rather
 * than assumed: the full-rate FP32 VALU issue rate, each transcendental, a
 * transcendental co-issued with FMAs, 32x32->64 products, int64 atomics in
 * global memory and in LDS at one address and at random addresses, and an
 * HBM stream (read, write, copy).
 *
 * Kernels run on the stream set by sde_set_stream (the null stream if none);
 * each call makes one untimed launch, then `reps` timed launches bracketed by
 * HIP events, and synchronises that stream before it returns.  Errors as in
 * sde.h; sde_last_error() explains.
 */
#ifndef SDE_ROOFS_H
#define SDE_ROOFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Kinds and their `variant`:
 *  SDE_MB_FMA     eight independent chains per lane of one full-rate VALU
 *                 operation: variant 0 v_fma_f32, 1 v_lshl_add_u32,
 *                 2 v_mul_f32, 3 v_add_f32, 4 v_xor_b32.
 *  SDE_MB_TRANS   one hardware transcendental, eight chains per lane;
 *                 variant 0 exp2, 1 log2, 2 rcp, 3 sqrt, 4 rsq, 5 sin.
 *  SDE_MB_MIX     four sqrt chains and 4 * variant FMA chains per lane,
 *                 variant in {1, 2, 4, 8}: whether transcendentals issue
 *                 beside FMAs (units: transcendentals + FMAs).
 *  SDE_MB_MUL64   32 x 32 -> 64-bit multiply-adds (v_mad_u64_u32, the
 *                 Philox round's product), eight chains per lane.
 *  SDE_MB_GATOMIC int64 add without return in global memory; variant 0: every
 *                 lane of the grid at one address, 1: each wave at its own
 *                 address (all its lanes there), 2: random addresses over the
 *                 largest power-of-two number of int64 words in `buf`.
 *  SDE_MB_LATOMIC int64 add without return in LDS (64 KiB per workgroup);
 *                 variant 0: one address per workgroup, 2: random addresses.
 *  SDE_MB_HBM     16-byte vector accesses over `buf`; variant 0 read, 1 write,
 *                 2 copy (first half to second half).  Units: bytes moved.
 */
enum {
    SDE_MB_FMA = 0,
    SDE_MB_TRANS = 1,
    SDE_MB_MIX = 2,
    SDE_MB_MUL64 = 3,
    SDE_MB_GATOMIC = 4,
    SDE_MB_LATOMIC = 5,
    SDE_MB_HBM = 6
};

/* Time one microbenchmark.
 *   kind, variant  as above.
 *   buf, buf_bytes device buffer owned by the caller (16-byte aligned); used
 *                  by SDE_MB_GATOMIC (>= 8 bytes, contents overwritten) and
 *                  SDE_MB_HBM (>= 1 MiB, a multiple of 32 bytes; read kinds
 *                  read whatever it holds); ignored otherwise (may be NULL).
 *   grid, block    launch shape: block a multiple of 64 in 64..1024, grid in
 *                  1..2^20.
 *   iters          per-lane iterations (1..2^24; ignored by SDE_MB_HBM,
 *                  which covers the buffer once per launch).
 *   reps           timed launches (1..100).
 *   units_out      work units of one launch (lane-operations, atomics or
 *                  bytes), exact.
 *   ms_out         mean duration of one timed launch in milliseconds.
 * Returns SDE_OK, SDE_E_INVALID for an unknown kind or variant or arguments
 * outside these ranges, SDE_E_HIP on a runtime failure. */
int sde_microbench(int kind, int variant, void* buf, size_t buf_bytes, int grid, int block,
                   int64_t iters, int reps, double* units_out, double* ms_out);

#ifdef __cplusplus
}
#endif

#endif /* SDE_ROOFS_H */
