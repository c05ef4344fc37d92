// Rigid pose from point correspondences by pairwise decoupling (Sec. 4.5).
//
//   k_pairs_count   one wave per row i: the pairs (i, j > i) that pass the
//                   length check of Sec. 4.5.1, counted by wave ballots
//   k_pairs_scan    exclusive scan of the row counts (one workgroup)
//   k_pairs_emit    the same test again; each kept pair written at its row's
//                   offset plus its rank among the row's kept pairs, so the
//                   output is in row order whatever the scheduling
//   k_t_keys        translation candidate t_i = y_i - R x_i and its cell
//                   (Sec. 4.5.2)
//   k_t_count       votes of each candidate's cell (the mode of the keys, by
//                   comparison against every key through LDS tiles; the key
//                   range split over the grid's second dimension)
//   k_t_best        the fullest cell, ties to the lowest index, by one 64-bit
//                   atomic max per workgroup
//   k_t_finish      the cell's centre
//   k_t_mask        |t_i - t|^2 <= T2 per correspondence, counted by ballots
//
// Every floating-point step is one binary32 operation in the order written
// (the library is compiled with -ffp-contract=off, '/' and sqrt correctly
// rounded), so the kept pairs, the cells and the inlier tests are
// reproducible bit for bit.
#include <algorithm>

#include "rv_device.h"
#include "rv_internal.h"
#include "rv_topk.h"

namespace rv {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kScanThreads = 1024;
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

// Length check of one pair: m = x_i - x_j, d = y_i - y_j, kept iff both
// lengths are nonzero and | |m| - |d| | <= mu (false for anything not finite).
__device__ __forceinline__ bool pair_kept(const float xi[3], const float yi[3], const float xj[3],
                                          const float yj[3], float mu, float m[3], float d[3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        m[c] = xi[c] - xj[c];
        d[c] = yi[c] - yj[c];
    }
    float sm = m[0] * m[0];
    sm = sm + m[1] * m[1];
    sm = sm + m[2] * m[2];
    float sd = d[0] * d[0];
    sd = sd + d[1] * d[1];
    sd = sd + d[2] * d[2];
    const float lm = __builtin_sqrtf(sm);
    const float ld = __builtin_sqrtf(sd);
    return (lm > 0.0f) && (ld > 0.0f) && (__builtin_fabsf(lm - ld) <= mu);
}

__device__ __forceinline__ void load3(const float* __restrict__ v, int64_t n, int64_t i, float o[3])
{
    o[0] = v[i];
    o[1] = v[n + i];
    o[2] = v[2 * n + i];
}

// A row's pairs are taken kRowUnroll vectors of 64 at a time: all their loads
// are issued before the first test, so the long rows (row i has n - 1 - i
// pairs, and the longest sets the kernel's duration) wait once per group
// instead of once per vector.  Loads past the last point read the last point
// and their pairs are not kept.
constexpr int kRowUnroll = 4;

// The wave's row (wave-uniform, held in scalar registers).
__device__ __forceinline__ int64_t wave_row()
{
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    return (int64_t)blockIdx.x * kWaves + w;
}

__global__ __launch_bounds__(kThreads) void k_pairs_count(const float* __restrict__ x,
                                                          const float* __restrict__ y, int64_t n,
                                                          float mu, uint64_t* __restrict__ rows)
{
    const int64_t i = wave_row();
    if (i >= n)
        return;
    const int lane = threadIdx.x & 63;
    float xi[3], yi[3];
    load3(x, n, i, xi);
    load3(y, n, i, yi);
    uint64_t cnt = 0;
    for (int64_t j0 = i + 1; j0 < n; j0 += 64 * kRowUnroll) {
        float xj[kRowUnroll][3], yj[kRowUnroll][3];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const int64_t j = j0 + u * 64 + lane;
            load3(x, n, j < n ? j : n - 1, xj[u]);
            load3(y, n, j < n ? j : n - 1, yj[u]);
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            float m[3], d[3];
            const bool keep = (j0 + u * 64 + lane < n) && pair_kept(xi, yi, xj[u], yj[u], mu, m, d);
            cnt += (uint64_t)__popcll(__ballot(keep));
        }
    }
    if (lane == 0)
        rows[i] = cnt;
}

// Exclusive scan in place; each thread scans a contiguous chunk.
__global__ __launch_bounds__(kScanThreads) void k_pairs_scan(uint64_t* __restrict__ rows, int64_t n,
                                                             RigidState* __restrict__ st)
{
    __shared__ uint64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    const int64_t b0 = (int64_t)t * per;
    const int64_t b = b0 < n ? b0 : n;
    const int64_t e = b + per < n ? b + per : n;
    uint64_t s = 0;
    for (int64_t i = b; i < e; ++i)
        s += rows[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint64_t add = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint64_t run = t ? part[t - 1] : 0ull;
    for (int64_t i = b; i < e; ++i) {
        const uint64_t c = rows[i];
        rows[i] = run;
        run += c;
    }
    if (t == kScanThreads - 1)
        st->pairs = part[t];
}

__global__ __launch_bounds__(kThreads) void k_pairs_emit(
    const float* __restrict__ x, const float* __restrict__ y, int64_t n, float mu,
    const uint64_t* __restrict__ rows, int64_t P, float* __restrict__ mo, float* __restrict__ no,
    int32_t* __restrict__ idx)
{
    const int64_t i = wave_row();
    if (i >= n)
        return;
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    float xi[3], yi[3];
    load3(x, n, i, xi);
    load3(y, n, i, yi);
    uint64_t k0 = rows[i];
    for (int64_t j0 = i + 1; j0 < n; j0 += 64 * kRowUnroll) {
        float xj[kRowUnroll][3], yj[kRowUnroll][3];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const int64_t j = j0 + u * 64 + lane;
            load3(x, n, j < n ? j : n - 1, xj[u]);
            load3(y, n, j < n ? j : n - 1, yj[u]);
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const int64_t j = j0 + u * 64 + lane;
            float m[3], d[3];
            const bool keep = (j < n) && pair_kept(xi, yi, xj[u], yj[u], mu, m, d);
            const uint64_t bal = __ballot(keep);
            if (keep) {
                const int64_t k = (int64_t)(k0 + (uint64_t)__popcll(bal & below));
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    mo[c * P + k] = m[c];
                    no[c * P + k] = d[c];
                }
                if (idx) {
                    idx[k] = (int32_t)i;
                    idx[P + k] = (int32_t)j;
                }
            }
            k0 += (uint64_t)__popcll(bal);
        }
    }
}

// R(q) of a unit quaternion, homogeneous form, row-major.
__device__ __forceinline__ void rotation_matrix(float w, float x, float y, float z, float R[9])
{
    const float ww = w * w, xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, xz = x * z, yz = y * z;
    const float wx = w * x, wy = w * y, wz = w * z;
    R[0] = (ww + xx) - (yy + zz);
    R[1] = 2.0f * (xy - wz);
    R[2] = 2.0f * (xz + wy);
    R[3] = 2.0f * (xy + wz);
    R[4] = (ww + yy) - (xx + zz);
    R[5] = 2.0f * (yz - wx);
    R[6] = 2.0f * (xz - wy);
    R[7] = 2.0f * (yz + wx);
    R[8] = (ww + zz) - (xx + yy);
}

struct TParams {
    float q[4];
    float t_min;
    float t_step;
    int t_cells;
    float T2;
};

// t_i = y_i - R x_i, (R x)_r = (R_r0 x_0 + R_r1 x_1) + R_r2 x_2.
__device__ __forceinline__ void t_candidate(const float* __restrict__ x, const float* __restrict__ y,
                                            int64_t n, int64_t i, const float R[9], float t[3])
{
    float xv[3], yv[3];
    load3(x, n, i, xv);
    load3(y, n, i, yv);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        float rx = R[3 * r] * xv[0];
        rx = rx + R[3 * r + 1] * xv[1];
        rx = rx + R[3 * r + 2] * xv[2];
        t[r] = yv[r] - rx;
    }
}

__device__ __forceinline__ uint32_t t_key(const float t[3], float t_min, float t_step, int T)
{
    const float fT = (float)T;
    uint32_t c[3];
    bool ok = true;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float u = (t[r] - t_min) / t_step;
        const bool in = (u >= 0.0f) && (u < fT);
        ok = ok && in;
        c[r] = in ? (uint32_t)u : 0u;
    }
    return ok ? (c[2] * (uint32_t)T + c[1]) * (uint32_t)T + c[0] : kNoKey;
}

__global__ void k_rigid_init(RigidState* __restrict__ st)
{
    if (threadIdx.x == 0) {
        st->best = 0ull;
        st->votes = 0ull;
        st->inliers = 0ull;
    }
}

__global__ __launch_bounds__(kThreads) void k_t_keys(const float* __restrict__ x,
                                                     const float* __restrict__ y, int64_t n,
                                                     TParams p, uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ votes)
{
    float R[9];
    rotation_matrix(p.q[0], p.q[1], p.q[2], p.q[3], R);
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        float t[3];
        t_candidate(x, y, n, i, R, t);
        keys[i] = t_key(t, p.t_min, p.t_step, p.t_cells);
        votes[i] = 0u;
    }
}

// Thread i counts, over the key range [blockIdx.y * span, +span), the keys
// equal to its own and adds that to votes[i] (zeroed by k_t_keys).
__global__ __launch_bounds__(kThreads) void k_t_count(const uint32_t* __restrict__ keys, int64_t n,
                                                      int64_t span, uint32_t* __restrict__ votes)
{
    __shared__ uint32_t tile[kThreads];
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const uint32_t mine = i < n ? keys[i] : kNoKey;
    const int64_t lo = (int64_t)blockIdx.y * span;
    const int64_t hi = lo + span < n ? lo + span : n;
    uint32_t cnt = 0;
    for (int64_t t0 = lo; t0 < hi; t0 += kThreads) {
        const int64_t j = t0 + threadIdx.x;
        tile[threadIdx.x] = j < hi ? keys[j] : kNoKey;
        __syncthreads();
        const int m = hi - t0 < kThreads ? (int)(hi - t0) : kThreads;
        for (int k = 0; k < m; ++k)
            cnt += tile[k] == mine ? 1u : 0u;
        __syncthreads();
    }
    if (i < n && mine != kNoKey && cnt)
        atomicAdd(votes + i, cnt);
}

// The fullest cell, ties to the lowest index: the maximum of
// (votes << 32 | ~key) over the candidates, one 64-bit atomic max per block.
__global__ __launch_bounds__(kThreads) void k_t_best(const uint32_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ votes, int64_t n,
                                                     RigidState* __restrict__ st)
{
    __shared__ uint64_t wbest[kWaves];
    uint64_t v = 0ull;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const uint32_t k = keys[i];
        if (k != kNoKey)
            v = umax64(v, ((uint64_t)votes[i] << 32) | (uint64_t)(~k));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = umax64(v, shfl_xor_u64(v, off));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (lane == 0)
        wbest[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t b = wbest[0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w)
            b = umax64(b, wbest[w]);
        if (b)
            atomicMax(reinterpret_cast<unsigned long long*>(&st->best), (unsigned long long)b);
    }
}

__global__ void k_t_finish(TParams p, RigidState* __restrict__ st)
{
    if (threadIdx.x != 0)
        return;
    const uint64_t b = st->best;
    if (b == 0ull) {
        st->t[0] = st->t[1] = st->t[2] = 0.0f;
        st->votes = 0ull;
        return;
    }
    const uint32_t key = ~(uint32_t)(b & 0xFFFFFFFFull);
    const uint32_t T = (uint32_t)p.t_cells;
    const uint32_t c[3] = {key % T, (key / T) % T, key / (T * T)};
#pragma unroll
    for (int r = 0; r < 3; ++r)
        st->t[r] = p.t_min + ((float)c[r] + 0.5f) * p.t_step;
    st->votes = b >> 32;
}

__global__ __launch_bounds__(kThreads) void k_t_mask(const float* __restrict__ x,
                                                     const float* __restrict__ y, int64_t n,
                                                     TParams p, uint8_t* __restrict__ mask,
                                                     RigidState* __restrict__ st)
{
    float R[9];
    rotation_matrix(p.q[0], p.q[1], p.q[2], p.q[3], R);
    const bool any = st->votes != 0ull;
    const float ts[3] = {st->t[0], st->t[1], st->t[2]};
    const int lane = threadIdx.x & 63;
    uint64_t cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t base = (int64_t)blockIdx.x * kThreads + (threadIdx.x & ~63); base < n;
         base += stride) {
        const int64_t i = base + lane;
        bool in = false;
        if (i < n) {
            float t[3];
            t_candidate(x, y, n, i, R, t);
            const float e0 = t[0] - ts[0], e1 = t[1] - ts[1], e2 = t[2] - ts[2];
            float d2 = e0 * e0;
            d2 = d2 + e1 * e1;
            d2 = d2 + e2 * e2;
            in = any && (d2 <= p.T2);
            mask[i] = in ? 1 : 0;
        }
        cnt += (uint64_t)__popcll(__ballot(in));
    }
    if (lane == 0 && cnt)
        atomicAdd(reinterpret_cast<unsigned long long*>(&st->inliers), (unsigned long long)cnt);
}

int grid_for(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 2048));
}

}  // namespace

hipError_t launch_pairs_count(const float* x, const float* y, int64_t n, float mu, uint64_t* rows,
                              RigidState* st, hipStream_t s)
{
    const int64_t nblk = (n + kWaves - 1) / kWaves;
    if (nblk > 0x7FFFFFFF)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pairs_count, dim3((unsigned)nblk), dim3(kThreads), 0, s, x, y, n, mu, rows);
    hipLaunchKernelGGL(k_pairs_scan, dim3(1), dim3(kScanThreads), 0, s, rows, n, st);
    return hipGetLastError();
}

hipError_t launch_pairs_emit(const float* x, const float* y, int64_t n, float mu,
                             const uint64_t* rows, int64_t P, float* m_out, float* n_out,
                             int32_t* idx_out, hipStream_t s)
{
    const int64_t nblk = (n + kWaves - 1) / kWaves;
    if (nblk > 0x7FFFFFFF)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pairs_emit, dim3((unsigned)nblk), dim3(kThreads), 0, s, x, y, n, mu, rows,
                       P, m_out, n_out, idx_out);
    return hipGetLastError();
}

hipError_t launch_translation(const float* x, const float* y, int64_t n, const float q[4],
                              float t_min, float t_step, int t_cells, float T2, uint32_t* keys,
                              uint8_t* mask, RigidState* st, hipStream_t s)
{
    TParams p{{q[0], q[1], q[2], q[3]}, t_min, t_step, t_cells, T2};
    hipLaunchKernelGGL(k_rigid_init, dim3(1), dim3(64), 0, s, st);
    if (n > 0) {
        const int64_t nblk = (n + kThreads - 1) / kThreads;
        if (nblk > 0x7FFFFFFF)
            return hipErrorInvalidValue;
        // split the key range so that the grid holds about 2048 workgroups
        const int64_t splits = std::max<int64_t>(1, std::min<int64_t>(nblk, 2048 / nblk));
        const int64_t span = ((n + splits - 1) / splits + kThreads - 1) / kThreads * kThreads;
        const int64_t ny = (n + span - 1) / span;
        uint32_t* votes = keys + n;
        hipLaunchKernelGGL(k_t_keys, dim3(grid_for(n)), dim3(kThreads), 0, s, x, y, n, p, keys,
                           votes);
        hipLaunchKernelGGL(k_t_count, dim3((unsigned)nblk, (unsigned)ny), dim3(kThreads), 0, s,
                           keys, n, span, votes);
        hipLaunchKernelGGL(k_t_best, dim3(grid_for(n)), dim3(kThreads), 0, s, keys, votes, n, st);
    }
    hipLaunchKernelGGL(k_t_finish, dim3(1), dim3(64), 0, s, p, st);
    if (n > 0)
        hipLaunchKernelGGL(k_t_mask, dim3(grid_for(n)), dim3(kThreads), 0, s, x, y, n, p, mask, st);
    return hipGetLastError();
}

}  // namespace rv
