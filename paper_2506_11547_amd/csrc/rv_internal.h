// Internal launch interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rv {

// Device-resident result of one solve, copied back once at the end.
struct Result {
    float q[4];
    int64_t count;
    int32_t winner;
    int32_t n_cand;
};

// Candidate buffers written by the top-K stage and read by rescoring.
struct Candidates {
    float4* q;          // [64] decoded cell centres
    int32_t* votes;     // [64] cell vote counts
    int32_t* idx;       // [64] cell indices
    uint32_t* inliers;  // [64] exact inlier counts (zeroed by the top-K stage)
    Result* result;
};

constexpr int kMaxTopK = 64;
constexpr int kTopkMaxBlocks = 256;

hipError_t launch_fill(int32_t* p, int64_t count, int32_t value, hipStream_t s);

// Global-atomic vote: one wave per (64 correspondences, sample chunk).
hipError_t launch_vote_global(const float* x, const float* y, int64_t n, int G, int J,
                              const float2* table, int32_t* hist, int chunk, hipStream_t s);

// Top-K over the grid: per-block sorted lists, then one merging block that
// also decodes the candidates and clears the inlier counters.
int topk_blocks(int64_t ncell);
hipError_t launch_topk_partial(const int32_t* hist, int64_t ncell, int nblocks,
                               uint64_t* partial, hipStream_t s);
hipError_t launch_topk_final(const uint64_t* partial, int nblocks, int K, int G,
                             const Candidates& c, hipStream_t s);

hipError_t launch_rescore(const float* x, const float* y, int64_t n, float T2,
                          const Candidates& c, hipStream_t s);
hipError_t launch_mask(const float* x, const float* y, int64_t n, float T2, const Candidates& c,
                       uint8_t* mask, hipStream_t s);

}  // namespace rv
