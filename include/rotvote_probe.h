/* librotvote_probe.so: test and measurement hooks beside the solver library.
 *
 * Not part of a solve.  The step hooks run one device step of the binary32
 * rule the solver uses (its sections: the circle basis of Sec. 4.1 and
 * App. A, the chart and cell of Sec. 4.3.1 and Alg. 1, the cell-centre
 * decode, the residual of App. D), one thread per element, so that tests can
 * compare each step with a CPU implementation bit for bit.  The ceiling hooks
 * time micro-benchmarks of the GPU's own limits for the benchmark's roofline.
 *
 * Conventions: every pointer is device memory owned by the caller unless
 * stated; n is an element count (n <= 0 does nothing and returns 0); calls are
 * synchronous (the null stream, then a device synchronisation).  Return value:
 * 0 on success, a HIP error code when a launch or the synchronisation fails,
 * -1 for an invalid argument or (ceiling hooks) a failed self-check. */
#ifndef ROTVOTE_PROBE_H
#define ROTVOTE_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* out[i] = 1 / in[i]: the solver's correctly rounded reciprocal for inputs
 * in [1, 2] when fast != 0 (hardware estimate and one Newton step), else
 * IEEE division.  float32 [n] each. */
int rvp_recip(const float *in, float *out, int64_t n, int fast);

/* q[i] = a[i] / b[i] and r[i] = sqrt(a[i]), the device's IEEE operations.
 * float32 [n] each. */
int rvp_div_sqrt(const float *a, const float *b, float *q, float *r, int64_t n);

/* The circle basis (u, v) of correspondence i (Sec. 4.1, App. A) after
 * normalising x_i and y_i.  x, y: float32 SoA [3][n]; u, v: float32 [n][4]
 * (w, x, y, z); ok: int32 [n], 1 when both vectors are usable. */
int rvp_basis(const float *x, const float *y, int64_t n, float *u, float *v, int *ok);

/* Cell index (x fastest, grid G per axis) of the quaternion q[i] after the
 * canonical sign and the chart (Sec. 4.3.1, Alg. 1).  q: float32 [n][4];
 * out: int32 [n]; fast selects the reciprocal as in rvp_recip. */
int rvp_cells(const float *q, int64_t n, int G, int *out, int fast);

/* Unit quaternion of the centre of cell idx[i] at grid G (the candidate
 * decode).  idx: int32 [n]; q: float32 [n][4]. */
int rvp_decode(const int *idx, int64_t n, int G, float *q);

/* Squared residual |L_i q|^2 of correspondence i against the one quaternion
 * q (float32 [4]) (App. D), or -1 for an unusable correspondence.
 * x, y: float32 SoA [3][n]; out: float32 [n]. */
int rvp_residual(const float *x, const float *y, int64_t n, const float *q, float *out);

/* The sample table of rot_vote_solve_noalloc, computed on the device: out[2j]
 * = cos(theta_j), out[2j + 1] = sin(theta_j), theta_j = ((2j + 1 - J) / J)
 * (pi / 2) in binary64 rounded to binary32 (Alg. 1's circle samples).
 * out: float32 [2 J]. */
int rvp_table(int J, float *out);

/* Ceiling micro-benchmarks.  Each allocates its own buffers, runs one untimed
 * and one timed launch (HIP events), checks what it can of the result, frees
 * everything and writes the rate to the host double.
 *
 * 32-bit FMA lane-operations per second: blocks x 256 threads, each running
 * iters x 8 independent FMA chains. */
int rvp_ceil_valu(int blocks, int iters, double *ops_per_s);

/* LDS atomic adds per second into a 128 KiB array: blocks x 1024 threads,
 * iters adds each, at random cells (random != 0) or bank-distinct cells. */
int rvp_ceil_lds_atomic(int blocks, int iters, int random, double *atomics_per_s);

/* Relaxed device-scope atomic adds per second into an int32 grid of `cells`
 * entries (a power of two, 64 .. 2^26): blocks x 256 threads, iters adds
 * each, at random cells or (contiguous != 0) a wave into 64 consecutive
 * cells.  The grid's total is checked. */
int rvp_ceil_global_atomic(int64_t cells, int blocks, int iters, int contiguous,
                           double *atomics_per_s);

/* Bytes read plus written per second by a device copy of `bytes` (a
 * multiple of 16). */
int rvp_ceil_copy(int64_t bytes, double *bytes_per_s);

/* Bytes read per second by a streaming read of `bytes` (a multiple of 16),
 * four independent 16-byte loads per thread and step. */
int rvp_ceil_read(int64_t bytes, double *bytes_per_s);

#ifdef __cplusplus
}
#endif

#endif /* ROTVOTE_PROBE_H */
