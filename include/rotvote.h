/*
 * rotvote — robust rotation estimation by quaternion-circle voting on one
 * MI355X (gfx950), as a C ABI.
 *
 * Method ("Linearly Solving Robust Rotation Estimation", arXiv 2506.11547):
 * the rotations that take x_i to y_i form a great circle of the unit
 * quaternion sphere (Sec. 4.1), the null space of the 4x4 constraint
 * L_i q = 0 (Lemma 1, App. D).  Each circle is sampled, the samples are
 * projected stereographically into the cube [-1,1]^3 cut into G^3 cells
 * (Sec. 4.3.1) and every sample adds one vote to its cell (Alg. 1).  The K
 * cells with the most votes (Alg. 1's peak; Sec. 4.4 keeps several peaks)
 * are rescored exactly by counting |L_i q| <= 2 sin(eps/2), i.e. the angle
 * between R(q) x_i and y_i is at most eps, and the best one is returned with
 * its inlier count and inlier mask.
 *
 * Conventions used throughout:
 *  - correspondences: float32 structure-of-arrays, x[3*n] = {x_0..x_{n-1}
 *    components 0, then components 1, then components 2}; same for y.  Only
 *    the direction is used; a vector whose squared norm is not a positive
 *    finite float is "unusable": it casts no vote and is never an inlier.
 *  - quaternions: (w, x, y, z), Hamilton convention, returned with w >= 0
 *    (first nonzero component positive).
 *  - vote grid: int32 [G][G][G], x fastest: idx = (iz*G + iy)*G + ix; cell
 *    (ix,iy,iz) covers the chart points p = q_vec / (1 + w) with
 *    (p_c + 1) G/2 in [i_c, i_c + 1).
 *  - J samples per circle: 0 in the config means J = 8 G.
 *  - every call runs on the handle's HIP stream; rot_vote_solve returns after
 *    that stream has finished the solve.
 *  - errors: a negative rv_status; the outputs are left untouched and
 *    rot_vote_last_error(h) describes the reason.  A handle is not
 *    thread-safe; several handles may coexist on one device.
 */
#ifndef ROTVOTE_H
#define ROTVOTE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rv_handle rv_handle;

typedef enum rv_status {
    RV_OK = 0,
    RV_EINVAL = -1,        /* an argument is out of range, NULL, or not device memory */
    RV_ENOMEM = -2,        /* device or pinned host allocation failed */
    RV_EDEVICE = -3,       /* the HIP runtime reported an error */
    RV_EUNSUPPORTED = -4,  /* valid but beyond the library's limits (n*J > 2^31-1) */
    RV_EAGAIN = -5,        /* server: the request queue is full; submit again later */
    RV_ETIMEDOUT = -6      /* server: the request did not finish within the wait */
} rv_status;

/* How the vote histogram is accumulated; every strategy yields the same
 * histogram bit for bit (integer additions commute). */
typedef enum rv_vote_strategy {
    RV_VOTE_AUTO = 0,      /* chosen per (G, n) from measurements */
    RV_VOTE_GLOBAL = 1,    /* run-coalesced atomics straight into the grid */
    RV_VOTE_BRICK = 2,     /* runs binned by brick, bricks accumulated in LDS (grid <= 384) */
    RV_VOTE_KEYS = 3       /* every sample a key, keys sorted by brick in LDS and stored in
                              brick order, bricks accumulated in LDS (grid <= 384); automatic
                              for J <= 2 G, where nearly every sample starts a new cell */
} rv_vote_strategy;

enum {
    RV_FLAG_TIMING = 1u,          /* record per-stage HIP events (rot_vote_get_timings) */
    RV_FLAG_BATCH_GRIDS = 2u,     /* keep every batch instance's vote grid (test hook) */
    RV_FLAG_KEEP_HISTOGRAM = 4u   /* write every solve's whole vote grid to the handle
                                     (rot_vote_get_histogram).  Without it the brick and
                                     key strategies keep only each brick's best cells,
                                     which is all the solve's results need */
};

enum {
    RV_MAX_TOPK = 64,
    RV_MAX_GRID = 1024,
    RV_NUM_STAGES = 6,
    RV_MAX_BATCH_GRID = 64,
    RV_MAX_REFINE_ROUNDS = 64,
    RV_MAX_T_CELLS = 1024,
    RV_MAX_RIGID_N = 1 << 18, /* point correspondences of the quadratic rigid stages */
    RV_BATCH_BUCKETS = 4,     /* instance-size buckets of a batch schedule: n < 512,
                                 512 <= n < 2048, 2048 <= n < 8192, n >= 8192 */
    RV_NOALLOC_MAX_GRID = 64,       /* rot_vote_solve_noalloc: largest G */
    RV_NOALLOC_MAX_SAMPLES = 4096   /* rot_vote_solve_noalloc: largest J */
};

typedef struct rv_config {
    int32_t device;              /* HIP device ordinal */
    void *stream;                /* hipStream_t to launch on; NULL = the null stream */
    int64_t max_n;               /* largest n a solve may pass (>= 0) */
    int32_t max_grid;            /* largest G a solve may pass, 1..RV_MAX_GRID */
    int32_t samples_per_circle;  /* J; 0 = 8*G per solve */
    int32_t topk;                /* K candidates rescored, 1..RV_MAX_TOPK */
    int32_t vote_strategy;       /* rv_vote_strategy */
    uint32_t flags;              /* RV_FLAG_* */
    int32_t max_batch;           /* largest B of rot_vote_solve_batch (0: no batches) */
    int32_t batch_brick_edge;    /* batches' LDS bricks: 16 or 32 cells a side; 0: measured
                                    by rot_vote_tune_batch, else 32 */
    int32_t reserved;            /* must be 0 */
    int64_t max_pairs;           /* pair buffers of rot_vote_solve_rigid, 0..max_n pairs
                                    (0: no rigid solves); 25 bytes each */
} rv_config;

/* Fills *cfg with: device 0, null stream, max_n 1<<20, max_grid 256, J = 8G,
 * K = 16, automatic vote strategy, no flags, no batches, no pair buffers. */
void rot_vote_default_config(rv_config *cfg);

/* Creates a handle on cfg->device and allocates all device scratch for the
 * config's maxima: the G^3 int32 grid (64 MiB at G = 256), the sample table,
 * top-K and result buffers.  The handle owns that memory until destroy.
 * *out is set only on success.  RV_EINVAL for a bad config, RV_ENOMEM when the
 * scratch does not fit, RV_EDEVICE for other runtime errors. */
rv_status rot_vote_create(rv_handle **out, const rv_config *cfg);

/* Releases the handle and its scratch (after its stream is idle).  NULL is a
 * no-op. */
rv_status rot_vote_destroy(rv_handle *h);

/* Reason for the handle's last error ("" if none); valid until the next call
 * on h.  A NULL handle yields the reason of the last failed call made without
 * a handle (rot_vote_create or rot_vote_solve_noalloc). */
const char *rot_vote_last_error(const rv_handle *h);

/* Rebinds the handle to another HIP stream (e.g. the caller's current one).
 * Work already enqueued on the old stream is ordered before the handle's
 * next work on the new one (an event recorded on the old stream, waited on
 * by the new), so the two never use the handle's scratch at once. */
rv_status rot_vote_set_stream(rv_handle *h, void *stream);

/* One robust solve (Alg. 1 voting, then exact rescoring of the top K cells).
 *   x, y          device pointers, float32 SoA [3][n] (see conventions); read only.
 *   n             number of correspondences, 0..max_n.
 *   grid          G, cells per axis of the vote cube, 1..max_grid.
 *   eps_rad       inlier angle threshold in radians, (0, pi].
 *   q_out         host float[4]: the winning cell centre as a unit quaternion.
 *   inlier_count  host: number of usable correspondences with angle <= eps.
 *   inlier_mask   device uint8[n]: 1 for those correspondences, else 0.
 * n == 0 returns q = (1,0,0,0), count 0.  No votes at all (every
 * correspondence unusable) gives the same.  RV_EUNSUPPORTED if n*J exceeds
 * 2^31-1 (int32 vote counts).  Synchronous on the handle's stream. */
rv_status rot_vote_solve(rv_handle *h, const float *x, const float *y, int64_t n, int32_t grid,
                         float eps_rad, float q_out[4], int64_t *inlier_count,
                         uint8_t *inlier_mask);

/* Result of rot_vote_solve_async, written to device memory (32 bytes,
 * 8-byte aligned). */
typedef struct rv_result {
    float q[4];     /* the winning cell centre as a unit quaternion (w, x, y, z) */
    int64_t count;  /* inlier count of q */
    int32_t winner; /* index of the winning candidate; -1 when nothing voted */
    int32_t n_cand; /* candidates rescored (at most K) */
} rv_result;

/* rot_vote_solve without waiting (the same Alg. 1 vote and exact rescoring):
 * enqueues the whole solve on the handle's stream and returns.
 *   result_device  device memory, one rv_result, 8-byte aligned.
 *   inlier_mask    device uint8[n], as for rot_vote_solve.
 * Both are written when the stream reaches them; the caller synchronises the
 * stream (or waits on an event recorded after the call) before reading them,
 * and keeps x, y, the mask and result_device alive until then.  The results
 * are bit for bit those of rot_vote_solve on the same input.  Calls on one
 * handle share its scratch and are ordered by its stream; do not rebind the
 * stream while solves are in flight.  No host synchronisation and no
 * allocation take place, except on the first solve at a new J (see
 * rot_vote_get_plan), which synchronises the stream to upload the sample
 * table: solve once at each J before capturing calls into a HIP graph.
 * Argument errors are reported at once (nothing is enqueued); device errors
 * surface at the caller's next synchronisation.  rot_vote_get_topk and
 * rot_vote_get_histogram synchronise the stream and then describe this solve. */
rv_status rot_vote_solve_async(rv_handle *h, const float *x, const float *y, int64_t n,
                               int32_t grid, float eps_rad, rv_result *result_device,
                               uint8_t *inlier_mask);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One solve
 * as rot_vote_solve_async gives it (the same results bit for bit, for the
 * same x, y, n, grid, J, K and eps), with no handle and no allocation of any
 * kind: no hipMalloc, hipFree or allocating library call.
 *   x, y, n, grid, eps_rad, inlier_mask   as rot_vote_solve.
 *   samples_per_circle  J; 0 means 8 * grid.
 *   topk          K candidates rescored, 1..RV_MAX_TOPK.
 *   stream        hipStream_t of the calling thread's current device (NULL:
 *                 the null stream); the call enqueues its kernels there and
 *                 returns without waiting.
 *   result_device device memory, one rv_result, 8-byte aligned; written
 *                 when the stream reaches it, as for rot_vote_solve_async.
 * Scratch: the vote grid, sample table, top-K lists and candidates live in
 * one fixed device array inside the library (about 1.1 MiB), which each GPU
 * the library runs on holds from the library's load until the process ends.
 * Every call on a GPU uses that GPU's array and leaves the last call's
 * contents in it (each call clears what it needs), so calls whose work
 * overlaps on one GPU (two streams, or two threads) race and give wrong
 * results: order them (one stream, or events).  Limits of the fixed array:
 * grid 1..RV_NOALLOC_MAX_GRID (64^3 int32 cells, 1 MiB) and J up to
 * RV_NOALLOC_MAX_SAMPLES; beyond them the call returns RV_EUNSUPPORTED.
 * The first call on a device looks the array's address up on that device
 * (hipGetSymbolAddress): make it before capturing calls into a graph.
 * Errors: a negative rv_status with nothing enqueued, the reason in
 * rot_vote_last_error(NULL); device errors surface at the caller's next
 * synchronisation. */
rv_status rot_vote_solve_noalloc(const float *x, const float *y, int64_t n, int32_t grid,
                                 int32_t samples_per_circle, int32_t topk, float eps_rad,
                                 void *stream, rv_result *result_device, uint8_t *inlier_mask);

/* Vote strategy chosen by measurement: times `reps` solves of this input
 * (after one untimed solve) with each strategy the handle supports at this
 * grid and remembers the fastest for the grid; later solves at that grid
 * with vote_strategy AUTO use it.  Every strategy gives the same histogram
 * and results bit for bit (Alg. 1's vote is a sum of integer counts), so
 * tuning changes speed only.
 *   mask_scratch   device uint8[n] written by the timed solves.
 *   strategy_out   host (may be NULL): RV_VOTE_GLOBAL, RV_VOTE_BRICK or RV_VOTE_KEYS.
 *   ms_out         host float[3] (may be NULL): mean wall time per solve of
 *                  {global, brick, keys} in ms; -1 for a strategy not available
 *                  or not timed (keys are timed only for J <= 4 G).
 * Needs n >= 1; reps in 1..1000. */
rv_status rot_vote_tune(rv_handle *h, const float *x, const float *y, int64_t n, int32_t grid,
                        float eps_rad, int32_t reps, uint8_t *mask_scratch, int32_t *strategy_out,
                        float ms_out[3]);

/* Several rotations from one vote (Alg. 1 returning several high peaks; one
 * cluster point per rotation motion in the scene).  The vote, top-K and decode
 * are rot_vote_solve's; every candidate gets its exact inlier set (the solve's
 * rescoring test).  Models are then chosen greedily: the candidate with the
 * most inliers not claimed by an earlier model (ties to the earlier
 * candidate) becomes the next model while that number is >= min_inliers; it
 * claims those inliers and suppresses every candidate within sep_rad of it
 * (|q_a . q_b| >= cos(sep_rad / 2), float32).  The first model is the single
 * solve's result (rot_vote_get_topk reports the candidates' total counts).
 *   max_models    1..topk;  sep_rad in [0, pi];  min_inliers >= 1.
 *   q_out         host float[4 * max_models] (w >= 0), counts host
 *                 int64[max_models] (claimed inliers), n_models host int32:
 *                 entries past *n_models are untouched.
 *   labels        device uint8[n]: 0 unclaimed, m + 1 claimed by model m.
 * Synchronous on the handle's stream. */
rv_status rot_vote_solve_multi(rv_handle *h, const float *x, const float *y, int64_t n,
                               int32_t grid, float eps_rad, int32_t max_models, float sep_rad,
                               int64_t min_inliers, float *q_out, int64_t *counts,
                               int32_t *n_models, uint8_t *labels);

/* Least-squares refinement on an inlier set (Sec. 4.2: the eigenvector of
 * Q^T Q with the smallest eigenvalue, Q stacking the two hyperplane normals
 * of every inlier's circle).  A round solves on the correspondences whose mask
 * entry is nonzero, then rescores the refined rotation (|L_i q|^2 <= T2, as a
 * solve does) into the mask; rounds repeat until a rescoring changes no mask
 * entry or max_rounds have run.  A round whose system is ill-posed (its two
 * smallest eigenvalues within 1e-6 * max(1, m) of each other, m the
 * correspondences used: one correspondence, parallel ones, none) keeps the
 * current rotation.  Normals, sums and the 4x4 eigenproblem are float64; the
 * rotation is returned rounded to float32 with w >= 0.
 *   q_io          host float[4]: in, the rotation kept by an ill-posed round
 *                 (typically a solve's q); out, the refined rotation.
 *   inlier_count  host int64: inliers of the returned rotation.
 *   inlier_mask   device uint8[n]: in, the inlier set of the first round (any
 *                 nonzero entry); out, the inliers of the returned rotation.
 *   max_rounds    1..RV_MAX_REFINE_ROUNDS; rounds_run (host, may be NULL)
 *                 receives the rounds that ran before convergence.
 * n = 0 returns q_io unchanged and count 0.  Synchronous on the handle's stream. */
rv_status rot_vote_refine(rv_handle *h, const float *x, const float *y, int64_t n, float eps_rad,
                          int32_t max_rounds, float q_io[4], int64_t *inlier_count,
                          uint8_t *inlier_mask, int32_t *rounds_run);

/* Rigid pose from point correspondences, step 1 (Sec. 4.5, the pairwise
 * constraint and the length check of Sec. 4.5.1): for i < j the differences
 * m = x_i - x_j, n = y_i - y_j satisfy R m = n under the rigid motion
 * y = R x + t, and a rotation keeps lengths, so a pair is kept iff
 * | |m| - |n| | <= mu and both lengths are nonzero (binary32 lengths
 * sqrt((c0*c0 + c1*c1) + c2*c2); a pair with a non-finite value is dropped).
 * Kept pairs are written in row order (i ascending, then j ascending).
 *   x, y          device float32 SoA [3][n] points (not directions).
 *   n             0..min(max_n, RV_MAX_RIGID_N) correspondences; the work is
 *                 n(n-1)/2 pair tests (RV_EUNSUPPORTED above RV_MAX_RIGID_N).
 *   mu            length tolerance >= 0, in the points' units.
 *   capacity      room of the outputs, in pairs.
 *   m_out, n_out  device float32 SoA [3][P] for the P kept pairs (component c
 *                 of pair k at c*P + k).
 *   idx_out       device int32 [2][P] (i then j), or NULL.
 *   pairs         host: P.
 * When P > capacity nothing is written but *pairs, and the call returns
 * RV_ENOMEM.  Synchronous on the handle's stream. */
rv_status rot_vote_pairs(rv_handle *h, const float *x, const float *y, int64_t n, float mu,
                         int64_t capacity, float *m_out, float *n_out, int32_t *idx_out,
                         int64_t *pairs);

/* Rigid pose, the translation vote (Sec. 4.5.2): with the rotation q fixed,
 * every correspondence gives a candidate t_i = y_i - R(q) x_i; the candidates
 * vote in cubic cells of edge t_step over [t_min, t_min + t_cells * t_step)^3
 * (cell floor((t_r - t_min) / t_step) per axis, index (c_z*T + c_y)*T + c_x; a
 * candidate outside the domain or not finite does not vote), and t is the
 * centre t_min + (c + 0.5) * t_step of the cell with the most candidates
 * (ties to the lowest index).  A correspondence is an inlier iff
 * |t_i - t| <= t_inlier.  R(q) is the homogeneous rotation matrix of the unit
 * quaternion, all in binary32.  With no vote, t = 0 and there is no inlier.
 *   q             host float[4] (w, x, y, z), unit.
 *   t_step > 0, t_cells 1..RV_MAX_T_CELLS, t_inlier >= 0.
 *   t_out         host float[3];  t_votes, inliers: host.
 *   inlier_mask   device uint8[n].
 * The vote costs O(n^2) comparisons (the mode of n cell indices), like the
 * pair stage it follows: n is at most RV_MAX_RIGID_N (RV_EUNSUPPORTED above).
 * Synchronous on the handle's stream. */
rv_status rot_vote_translation(rv_handle *h, const float *x, const float *y, int64_t n,
                               const float q[4], float t_min, float t_step, int32_t t_cells,
                               float t_inlier, float t_out[3], int64_t *t_votes, int64_t *inliers,
                               uint8_t *inlier_mask);

typedef struct rv_rigid_params {
    float mu;                 /* length tolerance of the pair check */
    float eps_rad;            /* rotation inlier angle of the pairs' rescoring, (0, pi] */
    int32_t grid;             /* rotation vote grid G, 1..max_grid */
    int32_t refine_rounds;    /* least-squares rounds on the pairs' inliers, 0..64 */
    float t_min;              /* translation domain [t_min, t_min + t_cells * t_step)^3 */
    float t_step;             /* translation cell edge, > 0 */
    int32_t t_cells;          /* cells per axis, 1..RV_MAX_T_CELLS */
    float t_inlier;           /* inlier distance of the final pose, >= 0 */
} rv_rigid_params;

typedef struct rv_rigid_result {
    float q[4];               /* rotation, w >= 0 */
    float t[3];               /* translation */
    int32_t refine_rounds_run;
    int64_t pairs;            /* pairs kept by the length check */
    int64_t rot_inliers;      /* pairs within eps_rad of q */
    int64_t t_votes;          /* candidates in the translation cell */
    int64_t inliers;          /* correspondences within t_inlier of (q, t) */
} rv_rigid_result;

/* Rigid pose (R, t) from point correspondences by pairwise decoupling
 * (Sec. 4.5): rot_vote_pairs into the handle's pair buffers, the rotation
 * solve (rot_vote_solve) on the kept pairs, refine_rounds of rot_vote_refine
 * on the pairs' inliers when refine_rounds > 0, then rot_vote_translation.
 * Each stage gives exactly what the separate calls give.
 *   inlier_mask   device uint8[n] (the translation stage's mask).
 * RV_EUNSUPPORTED if the handle has no pair buffers (max_pairs = 0); RV_ENOMEM
 * (with res->pairs set) if more than max_pairs pairs pass the length check.
 * Synchronous on the handle's stream. */
rv_status rot_vote_solve_rigid(rv_handle *h, const float *x, const float *y, int64_t n,
                               const rv_rigid_params *p, rv_rigid_result *res,
                               uint8_t *inlier_mask);

/* Many independent solves in one pass (Alg. 1 and the rescoring for each
 * instance; the instances share grid, J, K and eps).  Instance b is the
 * column range [offsets[b], offsets[b+1]) of the SoA arrays x and y, which
 * hold n = offsets[B] columns; each instance gets exactly the result a
 * separate rot_vote_solve on its columns would give.  The batch is planned on
 * the device (rot_vote_solve_batch_async); this call uploads the offsets,
 * runs it and reads the results back.
 *   offsets       host int64[B+1], offsets[0] = 0, nondecreasing, offsets[B] <= max_n.
 *   B             0..max_batch instances (0 is a no-op).
 *   grid          1..min(max_grid, RV_MAX_BATCH_GRID).
 *   q_out         host float[4*B]; inlier_count host int64[B];
 *   inlier_mask   device uint8[offsets[B]].
 * RV_EUNSUPPORTED if an instance's n*J exceeds 2^31-1 or the handle was
 * created without batches (max_batch = 0) or with vote_strategy global.
 * Synchronous on the handle's stream. */
rv_status rot_vote_solve_batch(rv_handle *h, const float *x, const float *y, const int64_t *offsets,
                               int32_t B, int32_t grid, float eps_rad, float *q_out,
                               int64_t *inlier_count, uint8_t *inlier_mask);

/* rot_vote_solve_batch without a host round trip (Sec. 4.3: every
 * correspondence's circle is voted independently, so the instances are data
 * parallel): the offsets are read on the device, where one kernel plans the
 * whole batch (each instance's brick size from its size bucket and the
 * handle's batch schedule, its work units of up to 512 correspondences, its
 * queue capacities and pool offsets), and every later kernel is launched for
 * upper bounds and skips what the plan left empty.  Nothing waits for the
 * host and nothing is allocated, so a batch can be captured into a HIP graph
 * and replayed on new offsets and new columns of the same arrays.
 *   x, y            device float32 SoA [3][n_cols]; n_cols 0..max_n.
 *   offsets_device  device int64[B+1]: offsets[0] = 0, nondecreasing,
 *                   offsets[B] <= n_cols, every instance's n*J <= 2^31-1.
 *   B               1..max_batch (0 is a no-op); grid as rot_vote_solve_batch.
 *   results_device  device rv_result[B], 8-byte aligned: instance b's q,
 *                   count, winner and candidates rescored.
 *   inlier_mask     device uint8[n_cols]; entries past offsets[B] are untouched.
 * Offsets that break their rules are detected on the device: every result
 * then has winner -2, count 0, q = (1,0,0,0), and no mask entry is written.
 * The first batch at a new J synchronises the stream to upload the sample
 * table (as rot_vote_solve_async does): run one before capturing.  The
 * handle's batch scratch is shared by its calls, which its stream orders;
 * rot_vote_get_batch_topk synchronises and then describes this batch. */
rv_status rot_vote_solve_batch_async(rv_handle *h, const float *x, const float *y, int64_t n_cols,
                                     const int64_t *offsets_device, int32_t B, int32_t grid,
                                     float eps_rad, rv_result *results_device,
                                     uint8_t *inlier_mask);

/* The batch schedule at a grid: the brick edge (16 or 32 cells) of the
 * instances in each size bucket (RV_BATCH_BUCKETS entries).  Results are the
 * same under every schedule; only the speed changes.  Set: RV_EINVAL when the
 * config fixes batch_brick_edge or an edge is not 16 or 32.  Get: the edges
 * in force (the config's, the schedule set, tuned or loaded, else 32). */
rv_status rot_vote_set_batch_schedule(rv_handle *h, int32_t grid, const int32_t *edges);
rv_status rot_vote_get_batch_schedule(rv_handle *h, int32_t grid, int32_t *edges);

/* The batch schedule chosen by measurement on this batch: starting from 32^3
 * bricks for every size bucket, each bucket that has instances here in turn
 * takes 16^3 bricks if the whole batch then runs faster (`reps` timed
 * batches after one untimed, per trial); the faster schedule is kept for
 * this grid.  Arguments as rot_vote_solve_batch; mask_scratch is its
 * inlier_mask.  edges_out (host int32[RV_BATCH_BUCKETS], may be NULL): the
 * schedule kept; ms_out (host float[RV_BATCH_BUCKETS + 1], may be NULL): the
 * mean batch time with 32^3 everywhere, then after trying each bucket at
 * 16^3 (-1 for a bucket without instances).  RV_EINVAL when the config fixes
 * batch_brick_edge. */
rv_status rot_vote_tune_batch(rv_handle *h, const float *x, const float *y, const int64_t *offsets,
                              int32_t B, int32_t grid, float eps_rad, int32_t reps,
                              uint8_t *mask_scratch, int32_t *edges_out, float *ms_out);

/* The choices made by measurement (rot_vote_tune's vote strategy per grid,
 * the batch schedules) in a JSON file keyed by (GPU architecture, grid, J,
 * instance-size bucket).  Save merges the handle's choices into the file
 * (entries of other keys are kept; written to path.tmp, then renamed).  Load
 * applies the file's entries for this GPU's architecture and the handle's J
 * at each grid; *applied (may be NULL) counts them.  RV_EINVAL for a file
 * that cannot be read or written or is not a tuning file. */
rv_status rot_vote_save_tuning(rv_handle *h, const char *path);
rv_status rot_vote_load_tuning(rv_handle *h, const char *path, int32_t *applied);

/* Test hook (RV_FLAG_BATCH_GRIDS): copies instance b's vote grid of the last
 * batch to the device buffer dst (grid^3 int32). */
rv_status rot_vote_get_batch_histogram(rv_handle *h, int32_t b, int32_t *dst_device);

/* Test hook: instance b's candidates of the last batch, as rot_vote_get_topk. */
rv_status rot_vote_get_batch_topk(rv_handle *h, int32_t b, int32_t *n_cand, int32_t *votes,
                                  int32_t *cell_idx, int64_t *inliers, int32_t *winner);

/* Test hook (RV_FLAG_KEEP_HISTOGRAM): copies the last solve's vote grid (G^3
 * int32, x fastest) to the device buffer dst.  RV_EINVAL before the first
 * solve and for a handle created without the flag. */
rv_status rot_vote_get_histogram(rv_handle *h, int32_t *dst_device);

/* Test hook: the last solve's candidates.  Writes *n_cand (<= K) and, for
 * k < *n_cand, the cell vote count, cell index and exact inlier count of
 * candidate k (ordered by votes desc, index asc) to host arrays of length K;
 * *winner is the position of the returned candidate (-1 if none). */
rv_status rot_vote_get_topk(rv_handle *h, int32_t *n_cand, int32_t *votes, int32_t *cell_idx,
                            int64_t *inliers, int32_t *winner);

/* Test hook: J and the vote strategy the last solve used. */
rv_status rot_vote_get_plan(rv_handle *h, int32_t *samples_per_circle, int32_t *vote_strategy);

/* With RV_FLAG_TIMING: device milliseconds of the last solve's stages,
 * measured with HIP events on the handle's stream; ms must hold
 * RV_NUM_STAGES floats:
 *   0 prepare  (global: clear the grid; brick: size the brick queues)
 *   1 vote     (sample every circle and accumulate or bin its votes)
 *   2 reduce   (global: per-block top-64 scan; brick: accumulate bricks in LDS,
 *               write the grid, per-brick list of the K best)
 *   3 top-K    (merge the lists, decode the K candidates)
 *   4 rescore  (exact inlier count of every candidate)
 *   5 mask     (winner, inlier mask, result record) */
rv_status rot_vote_get_timings(rv_handle *h, float *ms);

/* Device bytes the handle allocated at create (its whole footprint: a solve
 * allocates nothing). */
rv_status rot_vote_get_footprint(const rv_handle *h, int64_t *device_bytes);

/* ---------------------------------------------------------------- serving
 * A request server with admission by device-memory footprint.  A request's
 * footprint is the scratch its solve needs: the G^3 int32 vote grid (1, 8 or
 * 64 MiB at G = 64, 128, 256) and, for grids solved by the brick strategy,
 * a run pool sized for its n (rot_vote_server_request_bytes).  All of it
 * comes from one device arena of hbm_budget bytes allocated at create.  The
 * server admits the oldest queued request as soon as one of its `workers`
 * lanes (a thread with its own HIP stream, default priority, and handle) is
 * free and the footprint fits in the arena's free bytes; the lane runs it
 * (rot_vote_solve, then rot_vote_refine if asked) while the next requests
 * are admitted on other lanes, so work in flight is bounded by memory, and
 * many small requests run on the device beside a large one.  A finished
 * request returns its bytes to the arena at once.  Requests are admitted in
 * arrival order: one that does not fit yet holds back the ones behind it.
 * Continuous batching: an admitted request with grid <= RV_MAX_BATCH_GRID
 * and n <= batch_max_n (and no refinement) takes the queued requests of the
 * same grid and eps with it (oldest first, up to max_batch of them and max_n
 * columns in all), gathered into one rot_vote_solve_batch whose run pool and
 * gathered columns are its footprint.  A request's result does not depend on
 * where or with what it ran: every path gives exactly rot_vote_solve's
 * result.  Beyond max_queue waiting requests a submission returns
 * RV_EAGAIN; a request whose footprint exceeds the arena is refused with
 * RV_ENOMEM.  Times are seconds of the host's monotonic clock. */
typedef struct rv_server rv_server;

typedef struct rv_server_config {
    int32_t device;
    int32_t workers;             /* lanes: requests (or fused batches) run at once, 1..64 */
    int64_t max_n;               /* largest request (and largest batch, in columns) */
    int32_t max_grid;
    int32_t topk;                /* K of every solve */
    int32_t samples_per_circle;  /* 0: J = 8 * grid */
    int32_t max_batch;           /* requests fused into one batched solve; 0 or 1: never */
    int64_t batch_max_n;         /* requests with n up to this (and grid <= 64) may be fused */
    int64_t max_queue;           /* waiting requests before RV_EAGAIN */
    int64_t hbm_budget;          /* bytes of the scratch arena shared by the requests in
                                    flight; 0: room for `workers` requests of the largest size */
    int32_t reserved[4];         /* must be 0 */
} rv_server_config;

enum {
    RV_REQ_AFTER_STREAM = 1u  /* the request's kernels start after the work enqueued on
                                 rv_request.stream before the submission (the producer of
                                 x and y), through an event recorded at submit */
};

typedef struct rv_request {
    const float *x;              /* device float32 [3][n] SoA, as rot_vote_solve */
    const float *y;
    int64_t n;
    int32_t grid;
    float eps_rad;
    uint8_t *inlier_mask;        /* device uint8[n], written by the request */
    int32_t refine_rounds;       /* 0: none; else rot_vote_refine after the solve */
    uint32_t flags;              /* RV_REQ_* */
    void *stream;                /* hipStream_t for RV_REQ_AFTER_STREAM (NULL: null stream) */
} rv_request;

typedef struct rv_reply {
    float q[4];
    int64_t inlier_count;
    int32_t status;              /* the solve's rv_status */
    int32_t batched;             /* requests in its solve (1: alone) */
    int32_t worker;              /* the lane that ran it */
    int32_t refine_rounds_run;
    double t_submit, t_start, t_end;
    int64_t scratch_bytes;       /* arena bytes its solve held (shared when batched) */
} rv_reply;

/* Fills *cfg: device 0, 4 lanes, max_n 1<<20, max_grid 256, K 16, J = 8G,
 * max_batch 64, batch_max_n 65536, max_queue 1<<20, hbm_budget 0. */
void rot_vote_server_default_config(rv_server_config *cfg);
/* Creates the lanes and the arena; RV_ENOMEM if they do not fit. */
rv_status rot_vote_server_create(rv_server **out, const rv_server_config *cfg);
/* Serves the queued requests (admission resumes if paused), stops the lanes,
 * frees everything.  NULL is a no-op.  Replies not collected are dropped. */
rv_status rot_vote_server_destroy(rv_server *s);
/* Validates the request (as rot_vote_solve would) and queues it; *ticket
 * identifies it for rot_vote_server_wait.  The buffers must stay valid until
 * the reply is collected; the mask is complete when the reply is. */
rv_status rot_vote_server_submit(rv_server *s, const rv_request *req, uint64_t *ticket);
/* Waits up to timeout_ms (< 0: forever) for the request and collects its reply
 * (once).  RV_ETIMEDOUT leaves it pending. */
rv_status rot_vote_server_wait(rv_server *s, uint64_t ticket, int32_t timeout_ms, rv_reply *out);
/* Lanes and device bytes (lanes' own scratch plus the arena); requests queued
 * and in flight. */
rv_status rot_vote_server_stats(rv_server *s, int32_t *workers, int64_t *device_bytes,
                                int64_t *queued, int64_t *in_flight);
/* The arena's size, bytes held by requests in flight now and at most so far,
 * and the most requests in flight at once so far (any pointer may be NULL). */
rv_status rot_vote_server_memory(rv_server *s, int64_t *arena_bytes, int64_t *in_use,
                                 int64_t *peak_in_use, int64_t *peak_in_flight);
/* paused != 0 stops admitting (submissions still queue); 0 resumes. */
rv_status rot_vote_server_pause(rv_server *s, int32_t paused);
/* The footprint a request of n correspondences at this grid is admitted with
 * when it runs alone. */
rv_status rot_vote_server_request_bytes(rv_server *s, int64_t n, int32_t grid, int64_t *bytes);
const char *rot_vote_server_last_error(const rv_server *s);

#ifdef __cplusplus
}
#endif
#endif
