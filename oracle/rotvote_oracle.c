/*
 * CPU oracle for quaternion-circle rotation voting (Sec. 4.1-4.3, Alg. 1,
 * App. A, App. D of "Linearly Solving Robust Rotation Estimation").
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow and obviously correct: one loop per
 * step of the method, in the method's order, with no blocking, fusion or
 * reordering.  It shares no code with the HIP library.
 *
 * Arithmetic: every float operation below is one IEEE-754 binary32 operation,
 * round to nearest even.  The file is compiled with -ffp-contract=off, so the
 * only fused multiply-adds are the explicit fmaf() calls of the sampling and
 * chart steps; sqrtf and '/' are correctly rounded.  Precision is binary32
 * because the paper fixes none and the integer results (cells, votes, inlier
 * decisions) must be taken in the kernel's precision.  Step constants are
 * computed in binary64 and rounded once.
 */
#include "rotvote_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI_2
#define M_PI_2 1.57079632679489661923
#endif

/* ---- Step 0: constants ------------------------------------------------ */

/* Alg. 1 discretises alpha over [-pi, pi] uniformly; the circle point is
 * q(alpha) = q_b1 cos(alpha/2) + q_b2 sin(alpha/2) (Sec. 4.1).  With
 * theta = alpha/2 we take J midpoints theta_j = -pi/2 + pi (j + 1/2) / J, a
 * half-open, duplicate-free half circle (the other half is the antipode). */
void orc_tables(int32_t J, float *C, float *S)
{
    for (int32_t j = 0; j < J; ++j) {
        double th = ((double)(2 * j + 1 - J) / (double)J) * M_PI_2;
        C[j] = (float)cos(th);
        S[j] = (float)sin(th);
    }
}

/* |L q| = |R(q) a - b| = 2 sin(psi/2) for the angle psi between R(q)a and b,
 * so "psi <= eps" reads |L q|^2 <= 4 sin^2(eps/2). */
float orc_residual_bound(float eps_rad)
{
    double s = sin(0.5 * (double)eps_rad);
    return (float)(4.0 * s * s);
}

/* ---- Step 1: unit directions (Sec. 4.1 works with a, b on S^2) ---------- */

int32_t orc_normalise(const float v[3], float out[3])
{
    float s = v[0] * v[0];
    s = s + v[1] * v[1];
    s = s + v[2] * v[2];
    float nrm = sqrtf(s);
    if (!(nrm > 0.0f) || !isfinite(nrm))
        return 0;
    out[0] = v[0] / nrm;
    out[1] = v[1] / nrm;
    out[2] = v[2] / nrm;
    return 1;
}

void orc_normalise_pairs(const float *x, const float *y, int64_t n, float *a, float *b,
                         uint8_t *ok)
{
    for (int64_t i = 0; i < n; ++i) {
        float xi[3] = {x[i], x[n + i], x[2 * n + i]};
        float yi[3] = {y[i], y[n + i], y[2 * n + i]};
        float ai[3] = {0.0f, 0.0f, 0.0f}, bi[3] = {0.0f, 0.0f, 0.0f};
        int32_t good = orc_normalise(xi, ai) && orc_normalise(yi, bi);
        if (!good) {
            ai[0] = ai[1] = ai[2] = 0.0f;
            bi[0] = bi[1] = bi[2] = 0.0f;
        }
        for (int c = 0; c < 3; ++c) {
            a[c * n + i] = ai[c];
            b[c * n + i] = bi[c];
        }
        ok[i] = (uint8_t)good;
    }
}

/* ---- Step 2: circle basis ---------------------------------------------- */

/* App. A: q^T M q = b^T R(q) a with M symmetric, eigenvalues (1,1,-1,-1);
 * the circle {R(q) a = b} is the unit sphere of the +1 eigenspace, which every
 * column of (I + M) lies in.  The column k* with the largest diagonal entry of
 * M has squared norm 2 (1 + M_k*k*) >= 2 because trace M = 0, so the basis
 * needs no trigonometry and no threshold.  Entries of M:
 *   M_00 = a.b,  M_kk = 2 a_m b_m - a.b (k = m+1),  M_k0 = (a x b)_m,
 *   M_{n+1,m+1} = a_n b_m + a_m b_n (n != m).
 * For k* = 0 the column is (1 + cos th, sin th c) with c = a x b / |a x b|,
 * i.e. the paper's minimal-geodesic q_b1 up to scale.  The second basis vector
 * is q_b2 = (0, b) (x) q_b1 (Sec. 4.1): [-b.u_vec, u_w b + b x u_vec]. */
int32_t orc_circle_basis(const float a[3], const float b[3], float u[4], float v[4])
{
    float d = a[0] * b[0];
    d = d + a[1] * b[1];
    d = d + a[2] * b[2];
    float c[3];
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];

    float g[4];
    g[0] = d;
    for (int m = 0; m < 3; ++m)
        g[m + 1] = 2.0f * (a[m] * b[m]) - d;
    int32_t ks = 0;
    for (int k = 1; k < 4; ++k)
        if (g[k] > g[ks])
            ks = k;

    float up[4];
    if (ks == 0) {
        up[0] = 1.0f + g[0];
        up[1] = c[0];
        up[2] = c[1];
        up[3] = c[2];
    } else {
        int m = ks - 1;
        up[0] = c[m];
        for (int n = 0; n < 3; ++n) {
            if (n == m)
                up[n + 1] = 1.0f + g[ks];
            else
                up[n + 1] = a[n] * b[m] + a[m] * b[n];
        }
    }

    float r2 = up[0] * up[0];
    r2 = r2 + up[1] * up[1];
    r2 = r2 + up[2] * up[2];
    r2 = r2 + up[3] * up[3];
    float r = sqrtf(r2);
    for (int k = 0; k < 4; ++k)
        u[k] = up[k] / r;

    float bu = b[0] * u[1];
    bu = bu + b[1] * u[2];
    bu = bu + b[2] * u[3];
    v[0] = -bu;
    v[1] = u[0] * b[0] + (b[1] * u[3] - b[2] * u[2]);
    v[2] = u[0] * b[1] + (b[2] * u[1] - b[0] * u[3]);
    v[3] = u[0] * b[2] + (b[0] * u[2] - b[1] * u[1]);
    return ks;
}

/* ---- Steps 4-6 ---------------------------------------------------------- */

/* Step 4 (Sec. 4.3: q and -q are one rotation, keep the half sphere with its
 * equator): flip the sign unless the first nonzero component is positive. */
static void canonicalise(float q[4])
{
    int neg;
    if (q[0] != 0.0f)
        neg = q[0] < 0.0f;
    else if (q[1] != 0.0f)
        neg = q[1] < 0.0f;
    else if (q[2] != 0.0f)
        neg = q[2] < 0.0f;
    else
        neg = q[3] < 0.0f;
    if (neg)
        for (int k = 0; k < 4; ++k)
            q[k] = -q[k];
}

/* Step 5 (stereographic projection, Sec. 4.3.1): projecting from the pole
 * w = -1 maps the half sphere w >= 0 onto the unit ball, p = q_vec / (1 + w).
 * Step 6 (Alg. 1's accumulator: the cube [-1,1]^3 cut into G steps per axis):
 * t = (p + 1) G/2 is evaluated as t = fma(q_c, r H, H) with r = 1/(1 + w)
 * and H = G/2; the cell is floor(t) clamped to [0, G-1]. */
int32_t orc_cell_of(const float q[4], int32_t G, float qc[4], float t[3], int32_t ic[3])
{
    float h = (float)G * 0.5f;
    for (int k = 0; k < 4; ++k)
        qc[k] = q[k];
    canonicalise(qc);
    float den = 1.0f + qc[0];
    float r = 1.0f / den;
    float rh = r * h;
    for (int c = 0; c < 3; ++c) {
        t[c] = fmaf(qc[c + 1], rh, h);
        float f = floorf(t[c]);
        int32_t i;
        if (f < 0.0f)
            i = 0;
        else if (f > (float)(G - 1))
            i = G - 1;
        else
            i = (int32_t)f;
        ic[c] = i;
    }
    return (ic[2] * G + ic[1]) * G + ic[0];
}

/* Step 3: the j-th sample of the circle, q = cos(theta_j) u + sin(theta_j) v,
 * evaluated per component as fma(C_j, u_c, S_j * v_c). */
static void sample(const float u[4], const float v[4], float Cj, float Sj, float q[4])
{
    for (int c = 0; c < 4; ++c)
        q[c] = fmaf(Cj, u[c], Sj * v[c]);
}

int32_t orc_circle_cells(const float x[3], const float y[3], int32_t G, int32_t J,
                         int32_t *cells)
{
    float a[3], b[3], u[4], v[4], q[4], qc[4], t[3];
    int32_t ic[3];
    if (!orc_normalise(x, a) || !orc_normalise(y, b))
        return 0;
    orc_circle_basis(a, b, u, v);
    float *C = malloc(sizeof(float) * (size_t)J);
    float *S = malloc(sizeof(float) * (size_t)J);
    orc_tables(J, C, S);
    for (int32_t j = 0; j < J; ++j) {
        sample(u, v, C[j], S[j], q);
        cells[j] = orc_cell_of(q, G, qc, t, ic);
    }
    free(C);
    free(S);
    return 1;
}

/* ---- Step 7: Alg. 1's voting loop -------------------------------------- */

void orc_histogram(const float *x, const float *y, int64_t n, int32_t G, int32_t J,
                   int32_t *hist, int32_t nthreads)
{
    size_t ncell = (size_t)G * (size_t)G * (size_t)G;
    memset(hist, 0, ncell * sizeof(int32_t));
    float *C = malloc(sizeof(float) * (size_t)J);
    float *S = malloc(sizeof(float) * (size_t)J);
    orc_tables(J, C, S);
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i) {
        float xi[3] = {x[i], x[n + i], x[2 * n + i]};
        float yi[3] = {y[i], y[n + i], y[2 * n + i]};
        float a[3], b[3], u[4], v[4], q[4], qc[4], t[3];
        int32_t ic[3];
        if (!orc_normalise(xi, a) || !orc_normalise(yi, b))
            continue;
        orc_circle_basis(a, b, u, v);
        for (int32_t j = 0; j < J; ++j) {
            sample(u, v, C[j], S[j], q);
            int32_t idx = orc_cell_of(q, G, qc, t, ic);
#pragma omp atomic
            hist[idx] += 1;
        }
    }
    free(C);
    free(S);
}

/* ---- Step 8: top-K cells (Alg. 1 returns the highest block; Sec. 4.4
 * keeps several peaks) ---------------------------------------------------- */

int32_t orc_topk(const int32_t *hist, int32_t G, int32_t K, int32_t *counts, int32_t *idx)
{
    int64_t ncell = (int64_t)G * G * G;
    int32_t m = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        int32_t h = hist[c];
        if (h <= 0)
            continue;
        /* cells arrive in increasing idx, so among equal counts the earlier
         * entry already precedes: insert after every entry with count >= h */
        if (m == K && h <= counts[K - 1])
            continue;
        int32_t pos = m < K ? m : K - 1;
        while (pos > 0 && counts[pos - 1] < h) {
            counts[pos] = counts[pos - 1];
            idx[pos] = idx[pos - 1];
            --pos;
        }
        counts[pos] = h;
        idx[pos] = (int32_t)c;
        if (m < K)
            ++m;
    }
    return m;
}

/* ---- Step 9: cell centre back to S^3 (inverse projection, Sec. 4.3.1) ---- */

void orc_decode(int32_t idx, int32_t G, float q[4])
{
    int32_t ic[3];
    ic[0] = idx % G;
    ic[1] = (idx / G) % G;
    ic[2] = idx / (G * G);
    float p[3];
    for (int c = 0; c < 3; ++c)
        p[c] = (float)(2 * ic[c] + 1) / (float)G - 1.0f;
    float s = p[0] * p[0];
    s = s + p[1] * p[1];
    s = s + p[2] * p[2];
    float den = 1.0f + s;
    q[0] = (1.0f - s) / den;
    for (int c = 0; c < 3; ++c)
        q[c + 1] = (2.0f * p[c]) / den;
    canonicalise(q);
}

/* ---- Step 10: exact rescoring with the 4x4 constraint of App. D ---------- */

/* L(a,b) = [0, (a-b)^T; -(a-b), [a+b]_x]; L q = 0 is the circle (Lemma 1),
 * and |L q| = |R(q) a - b| for unit q. */
static float residual_unit(const float a[3], const float b[3], const float q[4])
{
    float D[3], P[3];
    for (int c = 0; c < 3; ++c) {
        D[c] = a[c] - b[c];
        P[c] = a[c] + b[c];
    }
    float w = q[0], vx = q[1], vy = q[2], vz = q[3];
    float r0 = D[0] * vx;
    r0 = r0 + D[1] * vy;
    r0 = r0 + D[2] * vz;
    float r1 = (P[1] * vz - P[2] * vy) - w * D[0];
    float r2 = (P[2] * vx - P[0] * vz) - w * D[1];
    float r3 = (P[0] * vy - P[1] * vx) - w * D[2];
    float s = r0 * r0;
    s = s + r1 * r1;
    s = s + r2 * r2;
    s = s + r3 * r3;
    return s;
}

float orc_residual(const float x[3], const float y[3], const float q[4])
{
    float a[3], b[3];
    if (!orc_normalise(x, a) || !orc_normalise(y, b))
        return -1.0f;
    return residual_unit(a, b, q);
}

int64_t orc_rescore(const float *x, const float *y, int64_t n, const float q[4], float T2,
                    uint8_t *mask)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        float xi[3] = {x[i], x[n + i], x[2 * n + i]};
        float yi[3] = {y[i], y[n + i], y[2 * n + i]};
        float a[3], b[3];
        int in = 0;
        if (orc_normalise(xi, a) && orc_normalise(yi, b))
            in = residual_unit(a, b, q) <= T2;
        cnt += in;
        if (mask)
            mask[i] = (uint8_t)in;
    }
    return cnt;
}

/* ---- Steps 0-11 ---------------------------------------------------------- */

int32_t orc_solve(const float *x, const float *y, int64_t n, int32_t G, int32_t J,
                  float eps_rad, int32_t K, int32_t nthreads, int32_t *hist,
                  int32_t *top_counts, int32_t *top_idx, int64_t *cand_counts,
                  float q_out[4], int64_t *count_out, int32_t *winner, uint8_t *mask)
{
    orc_histogram(x, y, n, G, J, hist, nthreads);
    int32_t m = orc_topk(hist, G, K, top_counts, top_idx);
    float T2 = orc_residual_bound(eps_rad);
    int32_t best = -1;
    int64_t best_cnt = -1;
    float best_q[4] = {1.0f, 0.0f, 0.0f, 0.0f};
    for (int32_t k = 0; k < m; ++k) {
        float q[4];
        orc_decode(top_idx[k], G, q);
        int64_t c = orc_rescore(x, y, n, q, T2, NULL);
        cand_counts[k] = c;
        if (c > best_cnt) {
            best_cnt = c;
            best = k;
            memcpy(best_q, q, sizeof best_q);
        }
    }
    memcpy(q_out, best_q, sizeof best_q);
    *winner = best;
    if (best < 0) {
        *count_out = 0;
        if (mask)
            memset(mask, 0, (size_t)n);
    } else {
        *count_out = orc_rescore(x, y, n, best_q, T2, mask);
    }
    return m;
}
