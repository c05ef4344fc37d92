/*
 * CPU oracle for quaternion-circle rotation voting.
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only users.  It shares no source with
 * the HIP library and the HIP library never calls it.
 *
 * Layout conventions: correspondences are float32 SoA [3][n] (x components,
 * then y, then z).  Quaternions are (w, x, y, z).  The vote grid is int32
 * [G][G][G] with x fastest: idx = (iz*G + iy)*G + ix.
 */
#ifndef ROTVOTE_ORACLE_H
#define ROTVOTE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Step 0: sample table (cos/sin of the half angles) and the residual bound. */
void orc_tables(int32_t J, float *C, float *S);
float orc_residual_bound(float eps_rad);

/* Step 1: returns 1 and writes the unit vector when the input is usable. */
int32_t orc_normalise(const float v[3], float out[3]);

/* Step 1 over SoA arrays [3][n]: unit a_i, b_i (zero when unusable) and the
 * usable flag of every correspondence. */
void orc_normalise_pairs(const float *x, const float *y, int64_t n, float *a, float *b,
                         uint8_t *ok);

/* Step 2: circle basis (u, v) of R q a = b; returns k*, the column used. */
int32_t orc_circle_basis(const float a[3], const float b[3], float u[4], float v[4]);

/* Steps 4-6 for one quaternion: canonical sign, chart, cell coordinates.
 * Writes the canonical quaternion, t (the scaled chart coordinates) and the
 * clamped integer cell coordinates; returns the linear cell index. */
int32_t orc_cell_of(const float q[4], int32_t G, float qc[4], float t[3], int32_t ic[3]);

/* Cells of every sample of one correspondence's circle (raw x_i, y_i, AoS [3]).
 * Returns 0 (and writes nothing) for an unusable correspondence. */
int32_t orc_circle_cells(const float x[3], const float y[3], int32_t G, int32_t J,
                         int32_t *cells);

/* Step 7 (Alg. 1): vote histogram over all correspondences.  hist has G^3
 * entries and is overwritten.  nthreads <= 1 runs single-threaded. */
void orc_histogram(const float *x, const float *y, int64_t n, int32_t G, int32_t J,
                   int32_t *hist, int32_t nthreads);

/* Step 8: the first min(K, #nonzero) cells by (count desc, idx asc). */
int32_t orc_topk(const int32_t *hist, int32_t G, int32_t K, int32_t *counts, int32_t *idx);

/* Step 9: cell centre -> canonical unit quaternion. */
void orc_decode(int32_t idx, int32_t G, float q[4]);

/* Step 10: squared constraint residual |L(a,b) q|^2 of one correspondence
 * (raw inputs); returns -1 for an unusable correspondence. */
float orc_residual(const float x[3], const float y[3], const float q[4]);

/* Step 10: inlier count of q over all correspondences; mask may be NULL. */
int64_t orc_rescore(const float *x, const float *y, int64_t n, const float q[4], float T2,
                    uint8_t *mask);

/* Steps 0-11: the whole solve.  hist (G^3) and the top-K arrays are outputs
 * too, so the tests can compare every intermediate.  Returns the number of
 * candidates; writes q, the winning count, the winner's position and mask. */
int32_t orc_solve(const float *x, const float *y, int64_t n, int32_t G, int32_t J,
                  float eps_rad, int32_t K, int32_t nthreads, int32_t *hist,
                  int32_t *top_counts, int32_t *top_idx, int64_t *cand_counts,
                  float q_out[4], int64_t *count_out, int32_t *winner, uint8_t *mask);

#ifdef __cplusplus
}
#endif
#endif
