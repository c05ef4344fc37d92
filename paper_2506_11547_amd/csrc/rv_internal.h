// Internal launch interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rotvote.h"

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
constexpr int kTopkMaxBlocks = 2048;  // also the largest brick count

hipError_t launch_fill(int32_t* p, int64_t count, int32_t value, hipStream_t s);

// Host helpers of the C-ABI layer: whether p is device (or managed) memory,
// and the rescoring bound 4 sin^2(eps / 2) rounded once to binary32.
bool is_device_memory(const void* p);
float residual_bound(float eps);
// Reason of the last failed call made without a handle (a create or the
// no-allocation solve), read by rot_vote_last_error(NULL); msg is a string
// literal (setting it allocates nothing).
void set_null_error(const char* msg);

// Global-atomic vote: one wave per (64 correspondences, sample chunk); chunk
// <= 0 picks chunks (whole table rows) for about 8192 waves.
hipError_t launch_vote_global(const float* x, const float* y, int64_t n, int G, int J,
                              const float2* table, int32_t* hist, int chunk, hipStream_t s);

// Top-K over the grid: per-block sorted lists, then one merging block that
// also decodes the candidates and clears the inlier counters.
int topk_blocks(int64_t ncell);
hipError_t launch_topk_partial(const int32_t* hist, int64_t ncell, int nblocks,
                               uint64_t* partial, hipStream_t s);
hipError_t launch_topk_final(const uint64_t* partial, int nblocks, int K, int G,
                             const Candidates& c, hipStream_t s);

// Brick-binned vote (G <= 256): estimate, plan, binned vote, brick accumulation.
constexpr int kQueueSets = 8;        // one queue per brick per XCD
constexpr int kMaxBricks = 512;      // (256 / 32)^3: bricks of a solve with 8-bit packed cells
constexpr int kNarrowGrid = 256;     // up to here cells pack 8 bits per axis, beyond 9
constexpr int kMaxBrickGrid = 384;   // (384 / 32)^3 = 1728 bricks
constexpr int kMaxBricksAll = 2048;  // brick tables of one solve (queue metadata, plan)
// The estimate samples every 64th correspondence, every 128th when runs are
// voted for 2^19 or more (each brick's estimate then still rests on thousands
// of sampled runs; keys, one per sample, keep the finer stride: their light
// bricks' estimates are too noisy at 128).
constexpr int kEstimateStride = 64;
inline int estimate_stride(int64_t n, bool keys)
{
    return (!keys && n >= ((int64_t)1 << 19)) ? 2 * kEstimateStride : kEstimateStride;
}

// A batch work unit: up to 512 consecutive correspondences of one instance
// (for the vote, the instance's index within its brick-size class).
struct Unit {
    int32_t inst;
    int32_t count;
    int64_t first;
};

// Queues are indexed [set][instance * nb + brick]: one solve uses kQueueSets
// sets (one per XCD) and qstride = kMaxBricksAll; a batch uses one set and
// qstride = B * nb.
struct BinArgs {
    uint32_t* pool;      // run queues; entry = narrow run: brick-local bits of bytes 1-3 and the
                         // length in byte 0; wide run: local cell | length << 15; key: the
                         // local cell in 16 bits (the pool read as uint16_t, same slot numbers)
    uint32_t* fill;      // [nsets][qstride] runs appended per queue
    uint32_t* qbase;     // [nsets][qstride] first pool slot of each queue
    uint32_t* cap;       // [qstride] capacity of each queue of the brick
    uint32_t* est;       // [kMaxBricksAll] estimated runs (sampled), zero between solves
    uint32_t* flags;     // [qstride] set when a brick's queue overflowed
    uint32_t* order;     // [kMaxBricksAll] one solve: bricks by decreasing capacity
    int32_t* ovf;        // [instances][G^3] overflow grids, zero between solves
    uint64_t pool_runs;  // pool capacity in runs (< 2^32)
    const Unit* units;   // batch: work units of the binned vote (null for one solve)
    const int32_t* counts;   // batch (device): [0] units, [1] instances of this launch's class
                             // (null: every launched block and `batch` instances)
    const int32_t* inst_of;  // batch (device): class-local instance -> batch instance, which
                             // indexes the overflow and kept grids (null: the same)
    int32_t nsets;
    int32_t qstride;
    int32_t batch;       // number of instances (0 for one solve)
};

// bricks per axis for bricks of 2^edge_log2 cells (4: 16, 5: 32)
int brick_axis(int G, int edge_log2);
// brick edge of a single solve at grid G: 16 up to G = 128 (at most 512
// bricks, enough workgroups for the accumulation), else 32
int solve_edge_log2(int G);
// estimate + plan (queue capacities); then the binned vote; then per-brick
// accumulation, which writes every cell of the grid and one sorted list per
// brick that holds the brick's K best cells.  Edge 16 needs G <= 256.
hipError_t launch_bin_prepare(const float* x, const float* y, int64_t n, int G, int J,
                              int edge_log2, const float2* table, const BinArgs& a, hipStream_t s,
                              bool keys = false);
// The key strategy's vote (32^3 bricks, every sample a key): after
// launch_bin_prepare(..., keys = true), before launch_brick_accum(edge 5).
hipError_t launch_key_vote(const float* x, const float* y, int64_t n, int G, int J,
                           const float2* table, const BinArgs& a, hipStream_t s);
hipError_t launch_bin_vote(const float* x, const float* y, int64_t n, int G, int J, int edge_log2,
                           const float2* table, const BinArgs& a, hipStream_t s);
// What the brick queues hold: narrow runs (G <= 256, the binned vote's), wide
// runs (the binned vote's above 256), or keys (the key vote's); edge 16 is
// narrow only.
enum class QueueFormat { kNarrow, kWide, kKeys };
hipError_t launch_brick_accum(int G, int K, int edge_log2, QueueFormat fmt, int32_t* grid,
                              uint64_t* partial, const BinArgs& a, hipStream_t s);

// Batches (G <= kMaxBatchGrid): planned on the device from the instances'
// offsets, then the binned vote over work units and the accumulation over
// (instance, brick), per brick-size class, then the per-instance top-K merge,
// rescore and mask.
constexpr int kMaxBatchGrid = 64;
constexpr int kMaxBatchBricks = 64;  // (64 / 16)^3
constexpr int kUnitSize = 512;       // correspondences per work unit
constexpr int kBatchBuckets = 4;     // instance-size buckets of a batch schedule
// Instance-size buckets: bucket k holds the instances with
// kBucketBound[k - 1] <= n < kBucketBound[k].
constexpr int64_t kBucketBound[kBatchBuckets - 1] = {512, 2048, 8192};

// Per-instance plan written by the plan kernel.
struct InstPlan {
    int32_t cls;      // brick-size class: 0 = 16^3 bricks, 1 = 32^3
    int32_t ci;       // index within the class
    int32_t unit0;    // first vote unit within the class
    int32_t gunit0;   // first unit of the batch-wide unit list
    int32_t nunits;
    uint32_t cap;     // run capacity of each of its queues
    uint32_t rbase;   // first pool slot of its queues
    int32_t reserved;
};

struct BatchPlanArgs {
    const int64_t* offsets;  // device int64[B + 1]
    int32_t B;
    int32_t J;
    int64_t n_cols;          // columns of the SoA input (offsets[B] must not exceed it)
    int8_t bucket_edge[kBatchBuckets];  // brick edge (log2) per instance-size bucket
    int32_t nb[2];           // bricks per instance of class 0 (16^3) and 1 (32^3)
    double share[2];         // planned runs per brick per correspondence, per class
    uint32_t slack[2];       // runs added to every queue, per class
    uint64_t pool_runs;
    InstPlan* inst;          // [B]
    int32_t* counts;         // [0..1] class 0 units, instances; [2..3] class 1; [4] all units;
                             // [5] 1 when the offsets are valid
    uint32_t* cap[2];        // per class: [instance in class * nb + brick]
    uint32_t* qbase[2];
    uint32_t* fill[2];
    uint32_t* flags[2];
    int32_t* inst_of[2];     // per class: class index -> batch instance
    Unit* units[2];          // per class: vote units (class-local instance)
    Unit* units_all;         // every unit (batch instance), for rescoring and masks
    Result* results;         // [B]: set for every instance when the offsets are invalid
};
// The plan (one workgroup) and its expansion into queues and units.
hipError_t launch_batch_plan(const BatchPlanArgs& p, hipStream_t s);

hipError_t launch_bin_vote_batch(const float* x, const float* y, int64_t n, int G, int J,
                                 int edge_log2, const float2* table, const BinArgs& a, int nunits,
                                 hipStream_t s);
// Per class: merge each instance's brick lists into its candidates (instances
// past counts[1] of the class skip).
hipError_t launch_batch_topk(const uint64_t* partial, int B, int nb, int K, int G,
                             const int32_t* counts, const int32_t* inst_of, const Candidates& c,
                             hipStream_t s);
// Rescore and mask over the batch's unit list (units past *nunits skip).
hipError_t launch_batch_rescore_mask(const float* x, const float* y, int64_t n, float T2,
                                     const Unit* units, int max_units, const int32_t* nunits,
                                     const int64_t* offsets, const Candidates& c, uint8_t* mask,
                                     hipStream_t s, hipEvent_t after_rescore);

// Least-squares refinement on an inlier set (Sec. 4.2): device-resident state
// of the rounds (rotation, counts, convergence), float64 block partials of the
// 10 distinct entries of sum_i M_i and the inlier count.
struct RefineState {
    float q[4];
    uint32_t done;        // the last round changed no mask entry
    uint32_t ill_posed;   // the last solve kept the previous rotation
    uint64_t count;       // inliers of the current rotation
    int64_t m;            // correspondences in the last solve
    int32_t rounds;       // rounds that ran (a converged round ends the rest)
    int32_t reserved;
};
constexpr int kRefineSums = 11;
constexpr int kRefineMaxBlocks = 1024;
constexpr double kRefineGapRel = 1e-6;  // ill-posed: two smallest eigenvalues this close (x max(1, m))
int refine_blocks(int64_t n);
hipError_t launch_refine(const float* x, const float* y, int64_t n, float T2, int rounds,
                         const float q_in[4], uint8_t* mask, RefineState* st, double* partial,
                         hipStream_t s);

// Several rotations from one vote: device state of the greedy model choice.
struct MultiState {
    unsigned long long counts[64];  // unclaimed inliers per candidate (running pass)
    uint64_t suppressed;            // candidates taken or within the separation angle
    int32_t n_models;
    uint32_t stop;                  // no further model
    int32_t m_cand[64];             // per model: candidate, claimed inliers, rotation
    int64_t m_count[64];
    float m_q[64][4];
};
hipError_t launch_multi(const float* x, const float* y, int64_t n, float T2, int max_models,
                        float cos_half_sep, int64_t min_inliers, const Candidates& c,
                        uint64_t* bits, uint8_t* labels, MultiState* st, hipStream_t s);

// Request staging of the server: separate requests' columns gathered into one
// batch array, the batch mask scattered back (units: inst = item, first =
// column within the item).
struct GatherItem {
    const float* x;
    const float* y;
    uint8_t* mask;
    int64_t n;
    int64_t offset;  // first column in the batch array
};
hipError_t launch_gather(const GatherItem* items, const Unit* units, int nunits, float* dx,
                         float* dy, int64_t total, hipStream_t s);
hipError_t launch_scatter_masks(const GatherItem* items, const Unit* units, int nunits,
                                const uint8_t* dmask, hipStream_t s);

// Rigid pose (Sec. 4.5): device state of the pair stage and the translation vote.
struct RigidState {
    uint64_t pairs;     // kept pairs (the row-count scan's total)
    uint64_t best;      // (votes << 32) | ~key of the fullest translation cell; 0: no vote
    float t[3];         // the cell's centre (0 without a vote)
    uint32_t reserved;
    uint64_t votes;
    uint64_t inliers;
};
// Pair stage: per-row counts of kept pairs into rows[0..n), their exclusive
// scan in place (total into st->pairs).
hipError_t launch_pairs_count(const float* x, const float* y, int64_t n, float mu, uint64_t* rows,
                              RigidState* st, hipStream_t s);
// Writes the P kept pairs at the scanned row offsets (row order).
hipError_t launch_pairs_emit(const float* x, const float* y, int64_t n, float mu,
                             const uint64_t* rows, int64_t P, float* m_out, float* n_out,
                             int32_t* idx_out, hipStream_t s);
// Translation vote, centre, inlier mask and count (keys: 2n uint32 scratch,
// the cells and their votes).
hipError_t launch_translation(const float* x, const float* y, int64_t n, const float q[4],
                              float t_min, float t_step, int t_cells, float T2, uint32_t* keys,
                              uint8_t* mask, RigidState* st, hipStream_t s);

hipError_t launch_rescore(const float* x, const float* y, int64_t n, float T2,
                          const Candidates& c, hipStream_t s);
// host_result (pinned host memory, or null): where the result record is also
// written, so a synchronous caller needs no device-to-host copy
hipError_t launch_mask(const float* x, const float* y, int64_t n, float T2, const Candidates& c,
                       uint8_t* mask, hipStream_t s, Result* host_result = nullptr);

// Server lanes: handles whose vote grid and run pool are not allocated at
// create but bound per solve from the server's arena.  The byte counts are
// what one solve (or one batch of B instances, `cols` columns in all) needs
// bound: the grid (global strategy) or grid + run pool (brick strategy), or
// the batch's run pool; -1 for arguments outside the handle's limits.
rv_status create_lane(rv_handle** out, const rv_config* cfg);
int64_t lane_solve_bytes(const rv_handle* h, int64_t n, int32_t grid);
int64_t lane_batch_bytes(const rv_handle* h, int64_t cols, int32_t B, int32_t grid);
void lane_bind(rv_handle* h, int32_t* grid, uint32_t* pool, uint64_t pool_runs);

}  // namespace rv
