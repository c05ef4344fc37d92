// Several rotations from one vote: the K candidates of the top-K stage, each
// with its exact inlier set, and a greedy choice of models (Alg. 1 returning
// several high peaks, one per rotation motion in the scene).  A model is the
// candidate with the most inliers that no earlier model claimed (ties to the
// earlier candidate), accepted while that number reaches min_inliers; it
// claims those inliers (label m + 1) and suppresses every candidate within
// the separation angle, |q_a . q_b| >= cos(sep / 2) in float32.
//
//   k_multi_bits     per correspondence, the 64-bit set of candidates it is an
//                    inlier of (the rule's residual test); total counts per
//                    candidate; labels cleared
//   k_multi_count    claim the previous model's inliers, then count each
//                    candidate's unclaimed inliers (one pass per model)
//   k_multi_pick     one wave: the next model, suppression, stop condition
#include <algorithm>

#include "rv_device.h"
#include "rv_internal.h"
#include "rv_topk.h"

namespace rv {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Each lane of a wave holds a per-candidate counter (lane k: candidate k);
// adds the wave's ballot of "bit k set" for every candidate k.
__device__ __forceinline__ void count_bits(uint64_t bits, int ncand, int lane, uint32_t& acc)
{
    for (int k = 0; k < ncand; ++k) {
        const uint32_t c = (uint32_t)__popcll(__ballot((bits >> k) & 1ull));
        acc += (lane == k) ? c : 0u;
    }
}

__device__ __forceinline__ void block_add_counts(uint32_t acc, uint32_t (*sh)[64], int ncand,
                                                 unsigned long long* out)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    sh[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && lane < ncand) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w)
            s += sh[w][lane];
        if (s)
            atomicAdd(out + lane, (unsigned long long)s);
    }
}

__global__ __launch_bounds__(kThreads) void k_multi_bits(const float* __restrict__ x,
                                                         const float* __restrict__ y, int64_t n,
                                                         float T2, Candidates c,
                                                         uint64_t* __restrict__ bits,
                                                         uint8_t* __restrict__ labels,
                                                         MultiState* __restrict__ st)
{
    __shared__ uint32_t sh[kWaves][64];
    const int lane = threadIdx.x & 63;
    const int ncand = __builtin_amdgcn_readfirstlane(c.result->n_cand);
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    // whole waves iterate together (the ballots need every lane)
    for (int64_t base = (int64_t)blockIdx.x * kThreads + (threadIdx.x & ~63); base < n;
         base += stride) {
        const int64_t i = base + lane;
        float a[3] = {1.0f, 0.0f, 0.0f}, b[3] = {1.0f, 0.0f, 0.0f};
        bool ok = false;
        if (i < n) {
            const bool oka = load_unit(x, n, i, a);
            const bool okb = load_unit(y, n, i, b);
            ok = oka && okb;
        }
        float D[3], P[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            D[m] = a[m] - b[m];
            P[m] = a[m] + b[m];
        }
        uint64_t mine = 0;
        for (int k = 0; k < ncand; ++k) {
            const float4 q4 = c.q[k];
            const Quat q{q4.x, q4.y, q4.z, q4.w};
            if (ok && residual2(D, P, q) <= T2)
                mine |= 1ull << k;
        }
        if (i < n) {
            bits[i] = mine;
            labels[i] = 0;
        }
        count_bits(mine, ncand, lane, acc);
    }
    block_add_counts(acc, sh, ncand, reinterpret_cast<unsigned long long*>(st->counts));
}

// Claims the inliers of the model picked last (if any), then counts every
// candidate's unclaimed inliers (count = false: claim only).
__global__ __launch_bounds__(kThreads) void k_multi_count(const uint64_t* __restrict__ bits,
                                                          uint8_t* __restrict__ labels, int64_t n,
                                                          Candidates c, MultiState* __restrict__ st,
                                                          int count)
{
    __shared__ uint32_t sh[kWaves][64];
    if (st->stop)
        return;
    const int lane = threadIdx.x & 63;
    const int ncand = __builtin_amdgcn_readfirstlane(c.result->n_cand);
    const int nm = st->n_models;               // models picked so far
    const int last = nm > 0 ? st->m_cand[nm - 1] : -1;
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t base = (int64_t)blockIdx.x * kThreads + (threadIdx.x & ~63); base < n;
         base += stride) {
        const int64_t i = base + lane;
        uint64_t free_bits = 0;
        if (i < n) {
            const uint64_t bi = bits[i];
            uint8_t lab = labels[i];
            if (lab == 0 && last >= 0 && ((bi >> last) & 1ull)) {
                lab = (uint8_t)nm;
                labels[i] = lab;
            }
            free_bits = lab == 0 ? bi : 0ull;
        }
        if (count)
            count_bits(free_bits, ncand, lane, acc);
    }
    if (count)
        block_add_counts(acc, sh, ncand, reinterpret_cast<unsigned long long*>(st->counts));
}

// float32 dot product in a fixed order, no contraction
__device__ __forceinline__ float dot4(const float4& a, const float4& b)
{
    float s = a.x * b.x;
    s = s + a.y * b.y;
    s = s + a.z * b.z;
    s = s + a.w * b.w;
    return s;
}

__global__ __launch_bounds__(64) void k_multi_pick(Candidates c, MultiState* __restrict__ st,
                                                   int max_models, float cos_half_sep,
                                                   int64_t min_inliers)
{
    if (st->stop)
        return;
    const int lane = threadIdx.x;
    const int ncand = c.result->n_cand;
    const int nm = st->n_models;
    const bool eligible = lane < ncand && !((st->suppressed >> lane) & 1ull);
    const uint64_t cnt = lane < ncand ? st->counts[lane] : 0ull;
    // most unclaimed inliers, ties to the earlier candidate
    uint64_t key = eligible ? (((cnt + 1ull) << 6) | (uint64_t)(63 - lane)) : 0ull;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1)
        key = umax64(key, shfl_xor_u64(key, m));
    if (nm == 0 && lane < ncand)
        c.inliers[lane] = (uint32_t)cnt;  // nothing claimed yet: the total counts
    st->counts[lane] = 0ull;              // for the next pass
    const int best = key ? 63 - (int)(key & 63ull) : -1;
    const int64_t best_cnt = key ? (int64_t)(key >> 6) - 1 : -1;
    if (best < 0 || best_cnt < min_inliers || nm >= max_models) {
        if (lane == 0) {
            st->stop = 1u;
            if (nm == 0) {  // no model: the result record of an empty solve
                Result* r = c.result;
                r->q[0] = 1.0f;
                r->q[1] = r->q[2] = r->q[3] = 0.0f;
                r->count = 0;
                r->winner = -1;
            }
        }
        return;
    }
    const float4 qb = c.q[best];
    bool sup = lane == best;
    if (lane < ncand)
        sup = sup || fabsf(dot4(c.q[lane], qb)) >= cos_half_sep;
    const uint64_t supm = __ballot(sup);
    if (lane == 0) {
        st->suppressed |= supm;
        st->m_cand[nm] = best;
        st->m_count[nm] = best_cnt;
        st->m_q[nm][0] = qb.x;
        st->m_q[nm][1] = qb.y;
        st->m_q[nm][2] = qb.z;
        st->m_q[nm][3] = qb.w;
        st->n_models = nm + 1;
        if (nm == 0) {  // the first model is also the solve's result record
            Result* r = c.result;
            r->q[0] = qb.x;
            r->q[1] = qb.y;
            r->q[2] = qb.z;
            r->q[3] = qb.w;
            r->count = best_cnt;
            r->winner = best;
        }
    }
}

__global__ void k_multi_init(MultiState* __restrict__ st)
{
    const int lane = threadIdx.x;
    if (lane < 64)
        st->counts[lane] = 0ull;
    if (lane == 0) {
        st->suppressed = 0ull;
        st->n_models = 0;
        st->stop = 0u;
    }
}

}  // namespace

hipError_t launch_multi(const float* x, const float* y, int64_t n, float T2, int max_models,
                        float cos_half_sep, int64_t min_inliers, const Candidates& c,
                        uint64_t* bits, uint8_t* labels, MultiState* st, hipStream_t s)
{
    const int64_t nwaves = (n + 63) / 64;
    const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>((nwaves + kWaves - 1) / kWaves, 2048));
    hipLaunchKernelGGL(k_multi_init, dim3(1), dim3(64), 0, s, st);
    hipLaunchKernelGGL(k_multi_bits, dim3(nblk), dim3(kThreads), 0, s, x, y, n, T2, c, bits, labels,
                       st);
    if (hipError_t e = hipGetLastError(); e != hipSuccess)
        return e;
    for (int m = 0; m < max_models; ++m) {
        if (m > 0)  // claim model m-1's inliers, count for model m
            hipLaunchKernelGGL(k_multi_count, dim3(nblk), dim3(kThreads), 0, s, bits, labels, n,
                               c, st, 1);
        hipLaunchKernelGGL(k_multi_pick, dim3(1), dim3(64), 0, s, c, st, max_models, cos_half_sep,
                           min_inliers);
        if (hipError_t e = hipGetLastError(); e != hipSuccess)
            return e;
    }
    // claim the last model's inliers
    hipLaunchKernelGGL(k_multi_count, dim3(nblk), dim3(kThreads), 0, s, bits, labels, n, c, st, 0);
    return hipGetLastError();
}

}  // namespace rv
