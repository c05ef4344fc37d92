// Least-squares refinement on an inlier set (Sec. 4.2): the rotation whose
// quaternion is the eigenvector of Q^T Q with the smallest eigenvalue, where Q
// stacks, for every inlier, the two unit normals of the hyperplanes that cut
// its circle out of S^3.  Those normals span the -1 eigenspace of M_i (App. A),
// so Q^T Q = sum_i (I - M_i) / 2: only the 10 distinct entries of sum_i M_i
// and the inlier count are accumulated (float64, from the float32 unit
// vectors; the products are exact), then one wave solves the 4x4 symmetric
// eigenproblem by cyclic Jacobi rotations in float64.  A round ends with the
// rule's rescoring of the refined rotation, which is the next round's inlier
// set; once a rescoring changes no mask entry the remaining rounds are no-ops
// (the same set gives the same rotation), decided on the device.
#include <algorithm>

#include "rv_device.h"
#include "rv_internal.h"

namespace rv {

namespace {

constexpr int kThreads = 256;
constexpr int kSums = kRefineSums;  // S00 S01 S02 S03 S11 S12 S13 S22 S23 S33, m

// M_i of App. A for unit a, b: q^T M q = b^T R(q) a.
//   M00 = a.b, M0k = (a x b)_m, Mkk = 2 a_m b_m - a.b, Mkl = a_m b_n + a_n b_m
__device__ __forceinline__ void add_m(const float a[3], const float b[3], double s[kSums])
{
    const double a0 = a[0], a1 = a[1], a2 = a[2];
    const double b0 = b[0], b1 = b[1], b2 = b[2];
    double dot = a0 * b0;
    dot = dot + a1 * b1;
    dot = dot + a2 * b2;
    s[0] += dot;
    s[1] += a1 * b2 - a2 * b1;
    s[2] += a2 * b0 - a0 * b2;
    s[3] += a0 * b1 - a1 * b0;
    s[4] += 2.0 * (a0 * b0) - dot;
    s[5] += a0 * b1 + a1 * b0;
    s[6] += a0 * b2 + a2 * b0;
    s[7] += 2.0 * (a1 * b1) - dot;
    s[8] += a1 * b2 + a2 * b1;
    s[9] += 2.0 * (a2 * b2) - dot;
    s[10] += 1.0;
}

// Block sum of kSums doubles in a fixed order (deterministic).
__device__ __forceinline__ void block_sum(double s[kSums], double (*sh)[kThreads])
{
#pragma unroll
    for (int k = 0; k < kSums; ++k)
        sh[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < kSums; ++k)
                sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void k_refine_accum(const float* __restrict__ x,
                                                           const float* __restrict__ y, int64_t n,
                                                           const uint8_t* __restrict__ mask,
                                                           const RefineState* __restrict__ st,
                                                           double* __restrict__ partial)
{
    __shared__ double sh[kSums][kThreads];
    if (st->done)
        return;
    double s[kSums];
#pragma unroll
    for (int k = 0; k < kSums; ++k)
        s[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        if (!mask[i])
            continue;
        float a[3], b[3];
        const bool oka = load_unit(x, n, i, a);
        const bool okb = load_unit(y, n, i, b);
        if (oka && okb)
            add_m(a, b, s);
    }
    block_sum(s, sh);
    if (threadIdx.x < kSums)
        partial[(int64_t)blockIdx.x * kSums + threadIdx.x] = sh[threadIdx.x][0];
}

// One cyclic Jacobi sweep on the symmetric 4x4 A (upper triangle used,
// kept symmetric), accumulating the rotations into V.
__device__ void jacobi_sweep(double A[4][4], double V[4][4])
{
    for (int p = 0; p < 3; ++p)
        for (int q = p + 1; q < 4; ++q) {
            const double apq = A[p][q];
            if (apq == 0.0)
                continue;
            // rotation angle that zeroes A[p][q]: t = tan(phi), the smaller root of
            // t^2 + 2 theta t - 1 = 0 with theta = (A_qq - A_pp) / (2 A_pq)
            const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0);
            const double sn = t * c;
            for (int k = 0; k < 4; ++k) {  // A <- A J (columns p, q)
                const double akp = A[k][p], akq = A[k][q];
                A[k][p] = c * akp - sn * akq;
                A[k][q] = sn * akp + c * akq;
            }
            for (int k = 0; k < 4; ++k) {  // A <- J^T A (rows p, q)
                const double apk = A[p][k], aqk = A[q][k];
                A[p][k] = c * apk - sn * aqk;
                A[q][k] = sn * apk + c * aqk;
            }
            A[p][q] = A[q][p] = 0.0;
            for (int k = 0; k < 4; ++k) {  // V <- V J
                const double vkp = V[k][p], vkq = V[k][q];
                V[k][p] = c * vkp - sn * vkq;
                V[k][q] = sn * vkp + c * vkq;
            }
        }
}

// The block partials summed in a fixed order (each thread a fixed subset,
// then a tree), then one thread solves the 4x4 eigenproblem.
__global__ __launch_bounds__(kThreads) void k_refine_solve(const double* __restrict__ partial,
                                                           int nblk, RefineState* __restrict__ st)
{
    __shared__ double sh[kSums][kThreads];
    if (st->done)
        return;
    double s[kSums];
#pragma unroll
    for (int k = 0; k < kSums; ++k)
        s[k] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads)
#pragma unroll
        for (int k = 0; k < kSums; ++k)
            s[k] += partial[(int64_t)b * kSums + k];
    block_sum(s, sh);
    if (threadIdx.x != 0)
        return;
    const double m = sh[10][0];
    // Q^T Q = (m I - S) / 2
    double A[4][4];
    const int idx[4][4] = {{0, 1, 2, 3}, {1, 4, 5, 6}, {2, 5, 7, 8}, {3, 6, 8, 9}};
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            A[r][c] = ((r == c ? m : 0.0) - sh[idx[r][c]][0]) * 0.5;
    double V[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    for (int sweep = 0; sweep < 32; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < 4; ++p) {
            diag += A[p][p] * A[p][p];
            for (int q = p + 1; q < 4; ++q)
                off += A[p][q] * A[p][q];
        }
        if (off <= 1e-40 * diag || off == 0.0)  // converged far below float64 resolution
            break;
        jacobi_sweep(A, V);
    }
    // the two smallest eigenvalues
    int k0 = 0;
    for (int k = 1; k < 4; ++k)
        if (A[k][k] < A[k0][k0])
            k0 = k;
    double second = 1e300;
    for (int k = 0; k < 4; ++k)
        if (k != k0 && A[k][k] < second)
            second = A[k][k];
    st->m = (int64_t)m;
    if (m == 0.0 || second - A[k0][k0] <= kRefineGapRel * fmax(1.0, m)) {
        st->ill_posed = 1u;  // keep the current rotation
        return;
    }
    double q[4] = {V[0][k0], V[1][k0], V[2][k0], V[3][k0]};
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    // canonical sign: w > 0, ties by the first nonzero component
    double sgn = 0.0;
    for (int k = 0; k < 4 && sgn == 0.0; ++k)
        if (q[k] != 0.0)
            sgn = q[k] > 0.0 ? 1.0 : -1.0;
    for (int k = 0; k < 4; ++k)
        st->q[k] = (float)(sgn * q[k] / nq);
    st->ill_posed = 0u;
}

// Rescoring of the refined rotation: the new mask, its count and the number of
// entries that changed.
__global__ __launch_bounds__(kThreads) void k_refine_mask(const float* __restrict__ x,
                                                          const float* __restrict__ y, int64_t n,
                                                          float T2, RefineState* __restrict__ st,
                                                          uint8_t* __restrict__ mask,
                                                          uint64_t* __restrict__ counts)
{
    __shared__ uint32_t sh_in[kThreads / 64], sh_ch[kThreads / 64];
    if (st->done)
        return;
    const Quat q{st->q[0], st->q[1], st->q[2], st->q[3]};
    uint32_t cin = 0, cch = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        float a[3], b[3];
        const bool oka = load_unit(x, n, i, a);
        const bool okb = load_unit(y, n, i, b);
        bool in = false;
        if (oka && okb) {
            float D[3], P[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                D[c] = a[c] - b[c];
                P[c] = a[c] + b[c];
            }
            in = residual2(D, P, q) <= T2;
        }
        const bool was = mask[i] != 0;
        mask[i] = in ? 1 : 0;
        cin += in ? 1u : 0u;
        cch += (in != was) ? 1u : 0u;
    }
    // wave sums, then one atomic per block
    for (int w = 32; w > 0; w >>= 1) {
        cin += __shfl_xor(cin, w);
        cch += __shfl_xor(cch, w);
    }
    if ((threadIdx.x & 63) == 0) {
        sh_in[threadIdx.x >> 6] = cin;
        sh_ch[threadIdx.x >> 6] = cch;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, c = 0;
        for (int w = 0; w < kThreads / 64; ++w) {
            a += sh_in[w];
            c += sh_ch[w];
        }
        // per-block counts, summed by k_refine_finish (no same-address
        // atomics from every XCD)
        counts[2 * blockIdx.x] = a;
        counts[2 * blockIdx.x + 1] = c;
    }
}

// End of a round: publish the count (the blocks' counts summed); a round that
// changed nothing marks the refinement as converged.
__global__ __launch_bounds__(kThreads) void k_refine_finish(RefineState* __restrict__ st,
                                                            const uint64_t* __restrict__ counts,
                                                            int nblk)
{
    __shared__ uint64_t sh[2][kThreads];
    if (st->done)
        return;
    const int t = threadIdx.x;
    uint64_t a = 0, c = 0;
    for (int b = t; b < nblk; b += kThreads) {
        a += counts[2 * b];
        c += counts[2 * b + 1];
    }
    sh[0][t] = a;
    sh[1][t] = c;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] += sh[0][t + w];
            sh[1][t] += sh[1][t + w];
        }
        __syncthreads();
    }
    if (t != 0)
        return;
    st->count = sh[0][0];
    st->rounds += 1;
    if (sh[1][0] == 0)
        st->done = 1u;
}

__global__ void k_refine_init(RefineState* __restrict__ st, float qw, float qx, float qy, float qz)
{
    if (threadIdx.x != 0)
        return;
    st->q[0] = qw;
    st->q[1] = qx;
    st->q[2] = qy;
    st->q[3] = qz;
    st->done = 0u;
    st->ill_posed = 0u;
    st->count = 0;
    st->m = 0;
    st->rounds = 0;
}

}  // namespace

int refine_blocks(int64_t n)
{
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kRefineMaxBlocks));
}

hipError_t launch_refine(const float* x, const float* y, int64_t n, float T2, int rounds,
                         const float q_in[4], uint8_t* mask, RefineState* st, double* partial,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_refine_init, dim3(1), dim3(64), 0, s, st, q_in[0], q_in[1], q_in[2],
                       q_in[3]);
    if (hipError_t e = hipGetLastError(); e != hipSuccess)
        return e;
    const int nblk = refine_blocks(n);
    for (int r = 0; r < rounds; ++r) {
        hipLaunchKernelGGL(k_refine_accum, dim3(nblk), dim3(kThreads), 0, s, x, y, n, mask, st,
                           partial);
        hipLaunchKernelGGL(k_refine_solve, dim3(1), dim3(kThreads), 0, s, partial, nblk, st);
        // the mask's per-block counts reuse the partial buffer (its sums are consumed)
        uint64_t* counts = reinterpret_cast<uint64_t*>(partial);
        hipLaunchKernelGGL(k_refine_mask, dim3(nblk), dim3(kThreads), 0, s, x, y, n, T2, st, mask,
                           counts);
        hipLaunchKernelGGL(k_refine_finish, dim3(1), dim3(kThreads), 0, s, st, counts, nblk);
        if (hipError_t e = hipGetLastError(); e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace rv
