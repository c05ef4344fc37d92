// Brick-binned vote for grids up to 384^3 (the grid is far larger than LDS and
// L2, so scattered atomics into it are bound by line traffic).
//
// The G^3 grid is cut into 32^3-cell bricks (128 KiB of int32, one brick per
// CU's LDS).  Each vote run (a cell and how many consecutive samples of one
// circle fell in it) is routed to its brick's queue in HBM; a second kernel
// accumulates each brick's queue in LDS and writes the finished brick out once,
// keeping its K best cells for the top-K stage.
//
//   k_bin_estimate  every 64th circle, runs counted per brick (queue sizing)
//   k_bin_plan      queue capacities and offsets in the run pool
//   k_vote_bin      all circles: sample, bin (LDS staging), append to queues
//   k_brick_accum   per brick: LDS histogram, write-out, sorted list of its K best
//
// Queues are kept per XCD (blockIdx % 8: workgroups are dispatched to the
// XCDs in turn), so a queue's tail is appended to from one XCD.  A queue that
// fills up sends its excess runs straight to a zeroed overflow grid with
// atomics, and the brick's accumulation adds (and re-zeroes) those cells: the
// capacities only change speed, never the histogram.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <type_traits>

#include "rv_device.h"
#include "rv_internal.h"
#include "rv_topk.h"

namespace rv {

namespace {

// Bricks are 2^kLog cells on a side: 32 (kLog 5, 128 KiB of LDS, one solve and
// batches) or 16 (kLog 4, 16 KiB, batches: many workgroups per CU).
template <int kLog>
struct Brick {
    static constexpr int kEdge = 1 << kLog;
    static constexpr int kCells = kEdge * kEdge * kEdge;
    static constexpr uint32_t kMask = (uint32_t)kEdge - 1u;
    static constexpr int kThreads = kLog == 5 ? 1024 : 256;  // accumulation workgroup
    static constexpr int kWaves = kThreads / kWave;
};
constexpr int kSets = kQueueSets;
typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // for non-temporal loads
constexpr int kStep = 8;  // samples between flush checks
// A staged run is its cell and its length: for G <= 256 the cell one byte
// per axis in bytes 1-3 and the length in byte 0 (runs cut every 240
// samples); for G <= 384 the cell 9 bits per axis with a 5-bit length above
// it (cut every 24 samples).  Cuts are multiples of 8 samples: the sample
// loop reads the table eight entries at a time.
template <bool kWide>
struct Pack {
    static constexpr int kBits = kWide ? 9 : 8;
    static constexpr uint32_t kAxis = (1u << kBits) - 1u;
    static constexpr int kLenShift = 3 * kBits;
    static constexpr uint32_t kCellMask = (1u << kLenShift) - 1u;
    static constexpr int kSplit = kWide ? 24 : 240;
    static_assert(kSplit % 8 == 0 && kSplit < (1 << (32 - kLenShift)), "cut and length field");
    static constexpr int kMaxBricksHere = kWide ? kMaxBricksAll : kMaxBricks;
    // Vote workgroups.  8-bit cells: 8 waves staging 1280 runs each keep a
    // workgroup's LDS at 48 KiB, so three share a CU (measured 7-10 % faster
    // than two with twice the staging).  9-bit cells: nearly every sample of
    // a short circle starts a run and 1728 bricks share a flush, so the runs
    // are stored in brick order (bin_flush_sorted): one 16-wave workgroup per
    // CU holds the staging and the 16-bit sort index (148 KiB of LDS).
    static constexpr int kWaves = kWide ? 16 : 8;
    static constexpr int kThreads = kWaves * kWave;
    static constexpr int kStageCap = 1280;
    static constexpr int kBlocksPerCU = kWide ? 1 : 3;
    // flush before a step could overflow a wave's staging: one step adds at
    // most kWave * kStep runs and a run-block boundary at most kWave more
    static constexpr int kFlushAt = kStageCap - kWave * kStep - kWave;
};
static_assert(Pack<false>::kThreads == kUnitSize, "a batch work unit is one vote block");
// Marks a dropped zero-length staged run.  A staged run never equals it: its
// length field is at most 240 (of 8 bits) or 24 (of 5 bits).
constexpr uint32_t kDropped = 0xFFFFFFFFu;
template <int kLog, bool kWide>
__device__ __forceinline__ uint32_t brick_of(uint32_t pc, int nba)
{
    using P = Pack<kWide>;
    const uint32_t ix = pc & P::kAxis, iy = (pc >> P::kBits) & P::kAxis,
                   iz = (pc >> (2 * P::kBits)) & P::kAxis;
    return __umul24(__umul24(iz >> kLog, (uint32_t)nba) + (iy >> kLog), (uint32_t)nba) +
           (ix >> kLog);
}

template <int kLog, bool kWide>
__device__ __forceinline__ uint32_t local_of(uint32_t pc)
{
    using P = Pack<kWide>;
    constexpr uint32_t m = Brick<kLog>::kMask;
    const uint32_t ix = pc & P::kAxis, iy = (pc >> P::kBits) & P::kAxis,
                   iz = (pc >> (2 * P::kBits)) & P::kAxis;
    return ((iz & m) << (2 * kLog)) | ((iy & m) << kLog) | (ix & m);
}

// Narrow staged runs (G <= 256): the cell one byte per axis in bytes 1-3
// (Cell::r8) and the run length in byte 0.  Their queue entries keep the
// brick-local coordinates in place (the low kLog bits of bytes 1-3) with the
// length: a mask, where the accumulation, which has ALU to spare, takes them
// apart.
// The brick of a narrow staged run: its brick coordinates, one per byte 1-3,
// weighted 1, nba and nba^2 by a byte dot product.  `weights` holds those
// bytes (brick_weights); nba^2 fits a byte since a narrow solve has at most
// 512 bricks.
__host__ __device__ constexpr uint32_t brick_weights(int nba)
{
    return (1u << 8) | ((uint32_t)nba << 16) | ((uint32_t)(nba * nba) << 24);
}
template <int kLog>
__device__ __forceinline__ uint32_t run_brick(uint32_t e, uint32_t weights)
{
    constexpr uint32_t kHigh = ((0xFFu >> kLog) << 8) | ((0xFFu >> kLog) << 16) | ((0xFFu >> kLog) << 24);
    return __builtin_amdgcn_udot4((e >> kLog) & kHigh, weights, 0u, false);
}
static_assert(kMaxBricks <= 512, "nba^2 <= 64 for narrow solves");
template <int kLog>
constexpr uint32_t kSpreadMask = (Brick<kLog>::kMask << 8) | (Brick<kLog>::kMask << 16) |
                                 (Brick<kLog>::kMask << 24) | 0xFFu;
template <int kLog>
__device__ __forceinline__ uint32_t spread_local(uint32_t e)
{
    // x + edge * y from bytes 1 and 2 by a byte dot product, plus z << 2 kLog
    constexpr uint32_t kWeights = (1u << 8) | ((uint32_t)Brick<kLog>::kEdge << 16);
    return __builtin_amdgcn_udot4(e, kWeights, (e >> 24) << (2 * kLog), false);
}

}  // namespace

// ------------------------------------------------------------- estimate

// Runs per brick of every stride-th correspondence.  One wave per
// (64 sampled correspondences, chunk of `chunk` samples, a multiple of 8), so
// the table index stays wave-uniform and the work spreads over the whole GPU.

template <int kLog, bool kWide, bool kKeys>
__global__ __launch_bounds__(256) void k_bin_estimate(const float* __restrict__ x,
                                                      const float* __restrict__ y, int64_t n,
                                                      float H, float gm, int J,
                                                      const float2* __restrict__ table, int nba,
                                                      int chunk, int ngroups, int nwaves,
                                                      int stride, uint32_t* __restrict__ est)
{
    __shared__ uint32_t s_est[Pack<kWide>::kMaxBricksHere];
    const int nb = nba * nba * nba;
    for (int b = threadIdx.x; b < nb; b += 256)
        s_est[b] = 0;
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (wave < nwaves) {
        const int c = wave / ngroups;
        const int g = wave - c * ngroups;
        const int64_t i = ((int64_t)g * kWave + (threadIdx.x & 63)) * stride;
        Quat u, v;
        const bool ok = load_circle(x, y, n, i, u, v);
        uint32_t cur = 0xFFFFFFFFu;
        for_samples<true>(u, v, table, c * chunk, min(J, (c + 1) * chunk), H, gm,
                          [&](const Cell& cell, int) {
                              const uint32_t pc = packed_coords<kWide>(cell);
                              // runs, or (keys) every sample
                              if (ok && (kKeys || pc != cur))
                                  atomicAdd(&s_est[brick_of<kLog, kWide>(pc, nba)], 1u);
                              cur = pc;
                          });
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += 256)
        if (s_est[b])
            atomicAdd(est + b, s_est[b]);
}

// ----------------------------------------------------------------- plan

// One block.  cap = 1.15 x the estimated runs of the brick spread over the
// queue sets, plus slack, in multiples of 64 runs (queues start 256-byte
// aligned); scaled down if the pool cannot hold them all; the bricks in
// decreasing order of capacity for the accumulation.  Resets the fill
// counters, the overflow flags and the estimate for the next solve.
constexpr int kPlanThreads = kMaxBricksAll / 2;  // two bricks per thread
constexpr int kPlanBuckets = 2 * kWave;          // capacity buckets of the accumulation order

__global__ __launch_bounds__(kPlanThreads) void k_bin_plan(BinArgs a, int nb, int stride)
{
    __shared__ uint64_t s_scan[kPlanThreads / kWave];
    __shared__ uint64_t s_total;
    __shared__ uint32_t s_hist[kPlanBuckets];
    const int t = threadIdx.x;
    const int b0 = 2 * t;  // this thread's bricks: b0 and b0 + 1
    uint64_t cap[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int b = b0 + h;
        if (b < nb) {
            const uint64_t e = (uint64_t)a.est[b] * (uint64_t)stride;
            cap[h] = ((e * 115 / 100) / kSets + 256 + 63) & ~63ull;
        }
    }
    // exclusive offsets of the bricks within one queue set: a scan over pairs
    // (shuffles within each wave, then over the wave totals)
    const int lane = t & (kWave - 1), wave = t / kWave;
    auto scan = [&](uint64_t& excl0, uint64_t& excl1) {
        const uint64_t v = cap[0] + cap[1];
        uint64_t incl = v;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint64_t w = __shfl_up(incl, off);
            incl += lane >= off ? w : 0ull;
        }
        if (lane == kWave - 1)
            s_scan[wave] = incl;
        __syncthreads();
        for (int w = 0; w < wave; ++w)
            incl += s_scan[w];
        if (t == kPlanThreads - 1)
            s_total = incl;
        __syncthreads();
        excl0 = incl - v;
        excl1 = excl0 + cap[0];
    };
    uint64_t excl0, excl1;
    scan(excl0, excl1);
    uint64_t total = s_total * kSets;
    if (total > a.pool_runs) {
        // proportional shrink, still in multiples of 64 runs
        const double f = (double)a.pool_runs / (double)total;
        cap[0] = (uint64_t)((double)cap[0] * f) & ~63ull;
        cap[1] = (uint64_t)((double)cap[1] * f) & ~63ull;
        __syncthreads();
        scan(excl0, excl1);
    }
    // accumulation order: heaviest bricks first, by a counting sort into
    // capacity buckets a quarter octave wide (largest first); within a bucket
    // the order is whichever the LDS atomics give.  The order only schedules
    // the accumulation (one workgroup per brick, handed out in order): any
    // order gives the same histogram.
    constexpr int kBuckets = kPlanBuckets;
    if (t < kBuckets)
        s_hist[t] = 0u;
    __syncthreads();
    int bk[2] = {0, 0};
    uint32_t pos[2] = {0u, 0u};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (b0 + h >= nb)
            continue;
        const uint64_t c = cap[h];
        int key = 0;  // 4 floor(log2 c) + the next two bits; c < 2^32
        if (c != 0) {
            const int l = 63 - __clzll((long long)c);
            key = 4 * l + (l >= 2 ? (int)((c >> (l - 2)) & 3u) : 0);
        }
        bk[h] = kBuckets - 1 - min(key, kBuckets - 1);
        pos[h] = atomicAdd(&s_hist[bk[h]], 1u);
    }
    __syncthreads();
    if (t < kWave) {
        // exclusive scan of the bucket counts, two buckets per lane, in place
        const uint32_t v0 = s_hist[2 * t], v1 = s_hist[2 * t + 1];
        uint32_t incl = v0 + v1;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t w = __shfl_up(incl, off);
            incl += t >= off ? w : 0u;
        }
        s_hist[2 * t] = incl - v0 - v1;
        s_hist[2 * t + 1] = incl - v1;
    }
    __syncthreads();
    const uint64_t excl[2] = {excl0, excl1};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int b = b0 + h;
        if (b >= nb)
            continue;
        a.order[s_hist[bk[h]] + pos[h]] = (uint32_t)b;
        a.cap[b] = (uint32_t)cap[h];
        for (int xs = 0; xs < kSets; ++xs) {
            a.qbase[xs * a.qstride + b] = (uint32_t)(xs * s_total + excl[h]);
            a.fill[xs * a.qstride + b] = 0u;
        }
        a.flags[b] = 0u;
        a.est[b] = 0u;
    }
}

// ------------------------------------------------------------ vote + bin

// Narrow staged runs (cell in bytes 1-3, length in byte 0).  Flush: runs
// counted per brick, one reservation atomic per brick, then each written to
// its queue slot as its spread brick-local cell and length (or, past the
// queue's capacity, added to the overflow grid).
template <int kLog>
__device__ __forceinline__ void bin_flush(uint32_t (*stage)[Pack<false>::kStageCap], uint32_t my,
                                          uint32_t* s_cnt, uint2* s_dst, int wave, int lane, int nb,
                                          int nba, int G, int xs, int qoff, int64_t ovf_off,
                                          const BinArgs& a)
{
    const uint32_t weights = brick_weights(nba);
    // (the loops step a wave-uniform base, so their counters are scalar)
    // 1: runs per brick (zero-length entries are marked dropped)
    for (uint32_t base = 0; base < my; base += kWave) {
        const uint32_t k = base + (uint32_t)lane;
        if (k < my) {
            const uint32_t e = stage[wave][k];
            if ((e & 0xFFu) == 0u)
                stage[wave][k] = kDropped;
            else
                atomicAdd(&s_cnt[run_brick<kLog>(e, weights)], 1u);
        }
    }
    __syncthreads();
    // 2: one reservation per brick in its queue; the first pool slot of this
    //    flush's runs and the room left before the queue's capacity
    for (int b = threadIdx.x; b < nb; b += Pack<false>::kThreads) {
        const uint32_t c = s_cnt[b];
        if (c) {
            const int64_t q = (int64_t)xs * a.qstride + qoff + b;
            const uint32_t g = atomicAdd(a.fill + q, c);
            const uint32_t cap = a.cap[qoff + b];
            s_dst[b] = make_uint2(a.qbase[q] + g, cap > g ? cap - g : 0u);
        }
    }
    __syncthreads();
    // 3: each run to its slot (brick recomputed from the staged entry).  Ranks
    //    count each brick's total back down to zero, so the counters are clear
    //    for the next flush once every wave is through here; the step barrier
    //    that precedes any flush guarantees that.
    for (uint32_t base = 0; base < my; base += 2 * kWave) {
        uint32_t ev[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t k = base + h * kWave + (uint32_t)lane;
            ev[h] = k < my ? stage[wave][k] : kDropped;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
        const uint32_t e = ev[h];
        if (e == kDropped)
            continue;
        const uint32_t b = run_brick<kLog>(e, weights);
        const uint32_t rank = atomicSub(&s_cnt[b], 1u) - 1u;
        // the destination and the room in one 64-bit LDS read
        const uint64_t d = *reinterpret_cast<const uint64_t*>(&s_dst[b]);
        const uint32_t slot = (uint32_t)d + rank;
        if (rank < (uint32_t)(d >> 32)) {
            a.pool[(uint64_t)slot] = e & kSpreadMask<kLog>;
        } else {
            const int64_t cell = ((int64_t)(e >> 24) * G + ((e >> 16) & 0xFFu)) * G + ((e >> 8) & 0xFFu);
            atomicAdd(a.ovf + ovf_off + cell, (int32_t)(e & 0xFFu));
            a.flags[qoff + b] = 1u;
        }
        }
    }
}

// The wide layout's flush: as bin_flush, but the runs are stored in brick
// order.  Phase 2 also gives every brick a block-local range of sorted
// positions (an exclusive scan of the counts), phase 3a puts each staged run's
// index at its position, and phase 3b stores the runs position by position,
// so a store instruction writes consecutive slots of a few bricks' queues
// instead of one slot in each of 64.
template <int kLog>
__device__ __forceinline__ void bin_flush_sorted(uint32_t (*stage)[Pack<true>::kStageCap],
                                                 uint32_t my, uint32_t* s_cnt, uint2* s_dst,
                                                 uint32_t* s_scan, uint16_t* s_idx,
                                                 uint32_t& s_total, int wave, int lane, int nb,
                                                 int nba, int G, int xs, int qoff,
                                                 int64_t ovf_off, const BinArgs& a)
{
    using P = Pack<true>;
    constexpr int kT = P::kThreads;
    constexpr int kPer = P::kMaxBricksHere / kT;
    static_assert(P::kWaves * P::kStageCap <= 65536, "16-bit sort index");
    static_assert(P::kMaxBricksHere % kT == 0, "every brick has a thread in the scan");
    const int t = threadIdx.x;
    // 1: runs per brick (zero-length entries are marked dropped)
    for (uint32_t k = lane; k < my; k += kWave) {
        const uint32_t e = stage[wave][k];
        if ((e >> P::kLenShift) == 0u) {
            stage[wave][k] = kDropped;
            continue;
        }
        atomicAdd(&s_cnt[brick_of<kLog, true>(e & P::kCellMask, nba)], 1u);
    }
    __syncthreads();
    // 2: each thread's bricks t*kPer.. (consecutive, so a scan of the
    //    per-thread sums orders the bricks); a reservation per brick, and the
    //    first sorted position of its runs in s_cnt.  The reservations (and
    //    the queues' capacities and bases) are requested here but first
    //    needed after the placement (3a), so their round trip overlaps the
    //    scan and the placement.
    uint32_t c[kPer], g[kPer], cap[kPer], qb[kPer];
    uint32_t sum = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int b = t * kPer + u;
        c[u] = b < nb ? s_cnt[b] : 0u;
        sum += c[u];
        const int64_t q = (int64_t)xs * a.qstride + qoff + b;
        g[u] = c[u] ? atomicAdd(a.fill + q, c[u]) : 0u;
        cap[u] = c[u] ? a.cap[qoff + b] : 0u;
        qb[u] = c[u] ? a.qbase[q] : 0u;
    }
    // inclusive scan of the sums within the wave, then over the wave totals
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off);
        incl += lane >= off ? v : 0u;
    }
    if (lane == kWave - 1)
        s_scan[wave] = incl;
    __syncthreads();
    uint32_t wpre = 0;
#pragma unroll
    for (int w = 0; w < P::kWaves; ++w)
        wpre += w < wave ? s_scan[w] : 0u;
    uint32_t pre = wpre + incl - sum;
    if (t == kT - 1)
        s_total = wpre + incl;
    uint32_t first[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int b = t * kPer + u;
        first[u] = pre;
        if (b < nb) {
            s_cnt[b] = pre;
            pre += c[u];
        }
    }
    __syncthreads();
    // 3a: each run's stage index at its sorted position (four runs per lane
    //     at a time, so their LDS round trips overlap)
    for (uint32_t k0 = lane; k0 < my; k0 += 4 * kWave) {
        uint32_t ev[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const uint32_t k = k0 + h * kWave;
            ev[h] = k < my ? stage[wave][k] : kDropped;
        }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            if (ev[h] == kDropped)
                continue;
            const uint32_t pos =
                atomicAdd(&s_cnt[brick_of<kLog, true>(ev[h] & P::kCellMask, nba)], 1u);
            s_idx[pos] = (uint16_t)(wave * P::kStageCap + k0 + h * kWave);
        }
    }
    // the bricks' destinations, now that their reservations are back (the
    // empty assembly statements keep the compiler from computing them, and
    // so waiting for the reservations, before the placement): the slot of
    // sorted position p is qbase + g + (p - first) (mod 2^32), positions
    // from first + room on overflow
#pragma unroll
    for (int u = 0; u < kPer; ++u)
        asm volatile("" : "+v"(g[u]), "+v"(cap[u]), "+v"(qb[u]));
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int b = t * kPer + u;
        if (b < nb && c[u]) {
            const uint32_t room = cap[u] > g[u] ? cap[u] - g[u] : 0u;
            s_dst[b] = make_uint2(qb[u] + g[u] - first[u], first[u] + min(room, c[u]));
        }
    }
    __syncthreads();
    // 3b: the runs in brick order; then the counters are cleared for the next
    //    flush (phase 3a is done everywhere, and a step barrier precedes it).
    //    The runs come from every wave's staging, so no wave may stage again
    //    before all are stored: the closing barrier.
    const uint32_t total = s_total;
    const uint32_t* flat = &stage[0][0];
    // four positions per thread at a time: their chains of LDS reads overlap
    for (uint32_t p0 = t; p0 < total; p0 += 4 * kT) {
        uint32_t ev[4], bv[4];
        uint2 dv[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const uint32_t p = p0 + h * kT;
            ev[h] = p < total ? flat[s_idx[p]] : 0u;
        }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            bv[h] = brick_of<kLog, true>(ev[h] & P::kCellMask, nba);
            dv[h] = s_dst[bv[h]];
        }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const uint32_t p = p0 + h * kT;
            if (p >= total)
                continue;
            const uint32_t pc = ev[h] & P::kCellMask;
            const uint32_t len = ev[h] >> P::kLenShift;
            const uint32_t b = bv[h];
            const uint2 d = dv[h];
            if (p < d.y) {
                a.pool[(uint64_t)(d.x + p)] = local_of<kLog, true>(pc) | (len << 15);
            } else {
                const int64_t cell = ((int64_t)((pc >> (2 * P::kBits)) & P::kAxis) * G +
                                      ((pc >> P::kBits) & P::kAxis)) * G + (pc & P::kAxis);
                atomicAdd(a.ovf + ovf_off + cell, (int32_t)len);
                a.flags[qoff + b] = 1u;
            }
        }
    }
    for (int b = t; b < nb; b += kT)
        s_cnt[b] = 0u;
    __syncthreads();
}

// One block per (512 correspondences, chunk of samples); chunks are whole run
// blocks, so splitting J across blocks only adds run boundaries.
template <int kLog, bool kWide>
__global__ __launch_bounds__(Pack<kWide>::kThreads, Pack<kWide>::kBlocksPerCU) void k_vote_bin(const float* __restrict__ x,
                                                              const float* __restrict__ y,
                                                              int64_t n, int G, float H, float gm,
                                                              int J, int chunk, int ngroups,
                                                              const float2* __restrict__ table,
                                                              int nba, BinArgs a)
{
    using P = Pack<kWide>;
    constexpr int kSplit = P::kSplit;
    __shared__ uint32_t stage[P::kWaves][P::kStageCap];
    __shared__ uint32_t s_cnt[P::kMaxBricksHere];
    __shared__ uint2 s_dst[P::kMaxBricksHere];
    // The flush decision: the largest staged count of the block's waves, by
    // an LDS atomic max into one of three slots used in turn.  Each check
    // clears the previous check's slot, which every wave has read before
    // this check's barrier and none writes again before the next barrier, so
    // every wave reads the same maximum and takes the same decision.
    __shared__ uint32_t s_maxfill[3];
    // the wide layout's per-wave scan totals, sort index and run total
    // (bin_flush_sorted)
    __shared__ uint32_t s_scan[P::kWaves];
    __shared__ uint16_t s_idx[kWide ? P::kWaves * P::kStageCap : 1];
    __shared__ uint32_t s_total;
    const int nb = nba * nba * nba;
    // a batch launched for an upper bound of its units: the rest return at once
    if (a.units && a.counts && (int)blockIdx.x >= a.counts[0])
        return;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int xs = a.nsets > 1 ? (int)(blockIdx.x & (kSets - 1)) : 0;
    int inst = 0, j0, j1;
    int64_t i0, iend;
    if (a.units) {  // batch: one unit of one instance, every sample
        const Unit un = a.units[blockIdx.x];
        inst = un.inst;
        i0 = un.first;
        iend = un.first + un.count;
        j0 = 0;
        j1 = J;
    } else {
        const int cb = blockIdx.x / ngroups;
        const int gb = blockIdx.x - cb * ngroups;
        i0 = (int64_t)gb * P::kThreads;
        iend = n;
        j0 = cb * chunk;
        j1 = min(J, j0 + chunk);
    }
    const int qoff = inst * nb;
    const int64_t ovf_off = (int64_t)(a.inst_of ? a.inst_of[inst] : inst) * G * G * G;
    for (int b = threadIdx.x; b < nb; b += P::kThreads) {
        s_cnt[b] = 0;
    }
    if (threadIdx.x < 3)
        s_maxfill[threadIdx.x] = 0u;
    __syncthreads();
    Quat u, v;
    const bool ok = load_circle(x, y, n, i0 + threadIdx.x, u, v) && (i0 + threadIdx.x < iend);
    uint32_t fill = 0;  // this wave's staged runs (wave-uniform)
    // The open run of each lane: its cell and length (narrow: `run`, the cell
    // in bytes 1-3 and the length in byte 0, kept as the staged entry itself).
    // A run is emitted when the cell changes and at every run-block end, where
    // its length restarts from 0; a block whose first sample leaves that cell
    // emits a zero-length entry, which the flush drops.  The first run starts
    // with a real cell of zero length for the same reason.
    uint32_t cur = 0u;
    uint32_t cnt = 0u;
    uint32_t run = 0u;
    uint32_t* my_stage = stage[wave];
    int slot = 0;

    // Emission without a branch: the ballot of the bare compare stays a
    // scalar mask (usable lanes are masked in the scalar domain), and the
    // staging store runs under that mask as the exec mask, narrowed and
    // restored around the one store in a single assembly block so that no
    // other instruction can be scheduled under it (the compiler, left to
    // branch, splits the emission into divergent blocks; a select between
    // the slot and a private dummy slot costs one instruction per sample).
    // The compiler does not count the block's store among the wave's LDS
    // operations; the waits for all of them that it puts before every barrier
    // are what order the store before the flush's reads (a CPU test checks
    // the compiled code for both that and the SCC clobber).
    const uint64_t okmask = __builtin_amdgcn_ballot_w64(ok);
    typedef __attribute__((address_space(3))) uint32_t lds_u32;
    auto emit = [&](bool change) {
        const uint64_t m = __builtin_amdgcn_ballot_w64(change) & okmask;
        const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        // the slot's LDS byte offset (the pointer converted to the LDS address space)
        const uint32_t addr = (uint32_t)(uintptr_t)(lds_u32*)(my_stage + fill + r);
        const uint32_t val = kWide ? cur | (cnt << P::kLenShift) : run;
        uint64_t save;
        asm volatile("s_and_saveexec_b64 %0, %1\n\tds_write_b32 %2, %3\n\ts_or_b64 exec, exec, %0"
                     : "=&s"(save)
                     : "s"(m), "v"(addr), "v"(val)
                     : "memory", "scc");
        fill += (uint32_t)__popcll(m);
    };

    auto flush = [&](uint32_t my) {
        if constexpr (kWide)
            bin_flush_sorted<kLog>(stage, my, s_cnt, s_dst, s_scan, s_idx, s_total, wave,
                                   lane, nb, nba, G, xs, qoff, ovf_off, a);
        else
            bin_flush<kLog>(stage, my, s_cnt, s_dst, wave, lane, nb, nba, G, xs, qoff,
                                   ovf_off, a);
    };

    for (int jb = j0; jb < j1; jb += kSplit) {
        const int je = min(j1, jb + kSplit);
        for (int js = jb; js < je; js += kStep) {
            for_samples<true>(u, v, table, js, min(je, js + kStep), H, gm, [&](const Cell& c, int) {
                if constexpr (kWide) {
                    const uint32_t pc = packed_coords<kWide>(c);
                    const bool change = pc != cur;
                    emit(change);
                    cnt = change ? 1u : cnt + 1u;
                    cur = change ? pc : cur;
                } else {
                    // the run grows by one sample, or a new one opens here
                    const bool change = c.r8 != cur;
                    emit(change);
                    run = (change ? c.r8 : run) + 1u;
                    cur = c.r8;
                }
            });
            if (lane == 0)
                atomicMax(&s_maxfill[slot], fill);
            __syncthreads();
            const bool need = s_maxfill[slot] > (uint32_t)P::kFlushAt;
            if (threadIdx.x == 0)
                s_maxfill[slot == 0 ? 2 : slot - 1] = 0u;
            if (need) {
                flush(fill);
                fill = 0;
            }
            slot = slot == 2 ? 0 : slot + 1;
        }
        emit(true);  // close every run at the block end (run lengths stay below 256)
        cnt = 0u;
        run &= ~0xFFu;
    }
    if (lane == 0)
        atomicMax(&s_maxfill[slot], fill);
    __syncthreads();
    if (s_maxfill[slot] > 0u)
        flush(fill);
}

// ------------------------------------------------------- vote by keys
//
// The key strategy, for circles sampled more sparsely than the grid's cells
// (J below about 2 G: nearly every sample lands in a new cell, so merging
// runs saves nothing and the run bookkeeping and the flush checks cost more
// than the samples).  Every sample is a key, brick index << 15 | cell within
// its 32^3 brick, written by every lane at a fixed slot (sample, lane) of its
// wave's staging, with no ballot or compaction; an unusable correspondence
// writes a dropped marker.  Each key is counted into its brick's LDS counter
// as it is staged (an atomic whose result is not waited for).  Every kWindow
// samples (the same sample index in every wave, so no flush check) the
// workgroup sorts its keys by brick in place (a counting sort in LDS: one
// reservation per brick and a scan of the counts give each brick's first
// position; every lane holds its staged keys in registers by then, and each
// key is written over the staging at the next free position of its brick's
// range, taken by an LDS atomic) and stores them position by position into
// the bricks' queues as 16-bit brick-local cells (one vote each), so one
// store instruction writes consecutive slots of a few bricks' queues.  The
// accumulation reads eight keys per 16-byte load and adds one per key.
template <int kWaves_, int kWindow_, int kBlocks_>
struct KeyPack {
    static constexpr int kWaves = kWaves_;
    static constexpr int kThreads = kWaves * kWave;
    static constexpr int kWindow = kWindow_;  // samples per flush, a multiple of 8
    static constexpr int kStageCap = kWindow * kWave;
    static constexpr int kBlocksPerCU = kBlocks_;
    static constexpr int kSplit = kWindow;    // chunks of J for few circles
    static_assert(kWindow % 8 == 0, "the sample loop reads the table eight entries at a time");
    static_assert(kMaxBricksAll % kThreads == 0, "every brick has a thread in the flush's scan");
};
// 16 waves in one workgroup per CU, flushing every 32 samples (2048 keys per
// wave; 152 KiB of LDS, the most a 16-wave window of 32-bit keys fits):
// larger flushes write longer stretches of each brick's queue and pay the
// barriers, the scan and the reservations less often.  Vote kernel measured
// at G = 360, J = 180: 0.427 ms, against 0.434 ms with 24-sample and 0.459 ms
// with 16-sample windows, and 0.452 and 0.556 ms with two 8-wave workgroups
// per CU (one flushing while the other samples) and 24- and 16-sample windows.
using Keys = KeyPack<16, 32, 1>;

constexpr uint32_t kKeyLocalBits = 15;  // cell within a 32^3 brick
constexpr uint32_t kKeyLocalMask = (1u << kKeyLocalBits) - 1u;
// The brick index sits above bit 16, so a key's low half-word is its cell
// (bit 15 clear) and is stored as it is.
constexpr uint32_t kKeyBrickShift = 16;

// Brick-axis weights of key_of for nba bricks per axis (under 2^24 for the
// 12 bricks per axis of G = 384).
__host__ __device__ constexpr uint32_t key_weight_y(uint32_t nba) { return nba * 65536u - 1024u; }
__host__ __device__ constexpr uint32_t key_weight_z(uint32_t nba) { return nba * nba * 65536u - 32768u; }
static_assert(key_weight_z(12) < (1u << 24), "24-bit multiplies");

// brick << 16 | cell within the brick, ((bz nba + by) nba + bx) << 16 |
// lz << 10 | ly << 5 | lx, as one sum over the axes: a coordinate v = 32 b + l
// at its cell weight w (1, 32, 1024) gives l w + 32 b w, and b times (brick
// weight - 32 w) completes the brick part (brick weights 65536, nba 65536,
// nba^2 65536); three 24-bit multiplies, no masks.
__device__ __forceinline__ uint32_t key_of(const Cell& c, uint32_t wy, uint32_t wz)
{
    static_assert(kKeyBrickShift == 16 && kKeyLocalBits == 15, "the weights assume this layout");
    return c.x + __umul24(c.x >> 5, 65536u - 32u) + (c.y << 5) + __umul24(c.y >> 5, wy) +
           (c.z << 10) + __umul24(c.z >> 5, wz);
}

template <class KP>
__device__ __forceinline__ void keys_flush(uint32_t (*stage)[KP::kStageCap], int nsamp,
                                           uint32_t* s_cnt, uint2* s_dst, uint32_t* s_scan,
                                           uint32_t& s_total,
                                           uint32_t (&ends)[kMaxBricksAll / KP::kThreads], int wave,
                                           int lane, int nb, int nba, int G, int xs,
                                           const BinArgs& a)
{
    constexpr int kT = KP::kThreads;
    constexpr int kPer = kMaxBricksAll / kT;
    const int t = threadIdx.x;
    uint32_t* const sorted = &stage[0][0];  // the sort's result, over every wave's staging
    // this wave's staged keys, into registers: the placement below writes
    // the sorted keys over the staging of all waves (every wave has read its
    // own before the second barrier)
    uint32_t ev[KP::kWindow];
#pragma unroll
    for (int h = 0; h < KP::kWindow; ++h)
        ev[h] = h < nsamp ? stage[wave][h * kWave + lane] : kDropped;
    // The keys were counted per brick as they were staged, on top of where
    // the previous flush's placement left each counter (its brick's end
    // position, kept in `ends` by the thread that owns the brick), so the
    // counters need no clearing between windows.
    __syncthreads();
    // The reservations (and the queues' capacities and bases) are requested
    // here but first needed after the placement (3a), so their round trip
    // overlaps the scan and the placement instead of stalling the workgroup.
    uint32_t c[kPer], g[kPer], cap[kPer], qb[kPer];
    uint32_t sum = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int b = t * kPer + u;
        c[u] = b < nb ? s_cnt[b] - ends[u] : 0u;
        sum += c[u];
        g[u] = c[u] ? atomicAdd(a.fill + (int64_t)xs * a.qstride + b, c[u]) : 0u;
        cap[u] = c[u] ? a.cap[b] : 0u;
        qb[u] = c[u] ? a.qbase[(int64_t)xs * a.qstride + b] : 0u;
    }
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off);
        incl += lane >= off ? v : 0u;
    }
    if (lane == kWave - 1)
        s_scan[wave] = incl;
    __syncthreads();
    uint32_t wpre = 0;
#pragma unroll
    for (int w = 0; w < KP::kWaves; ++w)
        wpre += w < wave ? s_scan[w] : 0u;
    uint32_t pre = wpre + incl - sum;
    if (t == kT - 1)
        s_total = wpre + incl;
    uint32_t first[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int b = t * kPer + u;
        first[u] = pre;
        if (b < nb) {
            s_cnt[b] = pre;  // the brick's first sorted position
            pre += c[u];
            ends[u] = pre;   // where placing the brick's keys leaves the counter
        }
    }
    __syncthreads();
    // 3a: each key to the next free position of its brick's range.  A
    //     lane's keys are all usable or all dropped (its correspondence's),
    //     and a group's positions are all taken before the first is used, so
    //     the compiler issues the group's atomics back to back and their LDS
    //     round trips overlap (a test per key would wait for each one).
    if (ev[0] != kDropped) {
        constexpr int kGroup = KP::kWindow % 16 == 0 ? 16 : 8;  // windows are multiples of 8
        if (nsamp == KP::kWindow) {
#pragma unroll
            for (int h0 = 0; h0 < KP::kWindow; h0 += kGroup) {
                uint32_t pos[kGroup];
#pragma unroll
                for (int h = 0; h < kGroup; ++h)
                    pos[h] = atomicAdd(&s_cnt[ev[h0 + h] >> kKeyBrickShift], 1u);
#pragma unroll
                for (int h = 0; h < kGroup; ++h)
                    sorted[pos[h]] = ev[h0 + h];
            }
        } else {  // the last window of a chunk (the tests on nsamp are uniform)
#pragma unroll
            for (int h0 = 0; h0 < KP::kWindow; h0 += kGroup) {
                uint32_t pos[kGroup];
#pragma unroll
                for (int h = 0; h < kGroup; ++h)
                    pos[h] = h0 + h < nsamp ? atomicAdd(&s_cnt[ev[h0 + h] >> kKeyBrickShift], 1u) : 0u;
#pragma unroll
                for (int h = 0; h < kGroup; ++h)
                    if (h0 + h < nsamp)
                        sorted[pos[h]] = ev[h0 + h];
            }
        }
    }
    // the bricks' destinations, now that their reservations are back (the
    // empty assembly statements keep the compiler from computing them, and
    // so waiting for the reservations, before the placement)
#pragma unroll
    for (int u = 0; u < kPer; ++u)
        asm volatile("" : "+v"(g[u]), "+v"(cap[u]), "+v"(qb[u]));
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int b = t * kPer + u;
        if (b < nb && c[u]) {
            const uint32_t room = cap[u] > g[u] ? cap[u] - g[u] : 0u;
            s_dst[b] = make_uint2(qb[u] + g[u] - first[u], first[u] + min(room, c[u]));
        }
    }
    __syncthreads();
    // 3b: each wave stores the sorted positions that lie in its own staging
    // area, so it goes on to stage the next window there without another
    // barrier; the next flush's first barrier keeps its writes of s_dst,
    // s_total and the sorted keys after these reads.
    const uint32_t total = s_total;
    const uint32_t lo = (uint32_t)wave * KP::kStageCap;
    const uint32_t hi = min(total, lo + (uint32_t)KP::kStageCap);
    // four positions per lane at a time: their LDS reads overlap
    constexpr int kU = 4;
    for (uint32_t p0 = lo + lane; p0 < hi; p0 += kU * kWave) {
        uint32_t sv[kU];
        uint2 dv[kU];
#pragma unroll
        for (int h = 0; h < kU; ++h) {
            const uint32_t p = p0 + h * kWave;
            sv[h] = p < hi ? sorted[p] : 0u;
        }
#pragma unroll
        for (int h = 0; h < kU; ++h)
            dv[h] = s_dst[sv[h] >> kKeyBrickShift];
        // a whole group of positions with room in every queue (the usual
        // case) is stored without a test per position
        const bool whole = p0 - lane + kU * kWave <= hi;
        bool spill = false;
#pragma unroll
        for (int h = 0; h < kU; ++h)
            spill |= p0 + h * kWave >= dv[h].y;
        if (whole && !__any(spill)) {
#pragma unroll
            for (int h = 0; h < kU; ++h)
                reinterpret_cast<uint16_t*>(a.pool)[(uint64_t)(dv[h].x + p0 + h * kWave)] = (uint16_t)sv[h];
            continue;
        }
#pragma unroll
        for (int h = 0; h < kU; ++h) {
            const uint32_t p = p0 + h * kWave;
            if (p >= hi)
                continue;
            const uint32_t e = sv[h];
            const uint32_t b = e >> kKeyBrickShift;
            const uint2 d = dv[h];
            if (p < d.y) {
                reinterpret_cast<uint16_t*>(a.pool)[(uint64_t)(d.x + p)] = (uint16_t)e;
            } else {
                const uint32_t l = e & kKeyLocalMask;
                const uint32_t bx = b % (uint32_t)nba, by = (b / (uint32_t)nba) % (uint32_t)nba,
                               bz = b / (uint32_t)(nba * nba);
                const int64_t cell = ((int64_t)(bz * 32 + (l >> 10)) * G + (by * 32 + ((l >> 5) & 31u))) * G +
                                     (bx * 32 + (l & 31u));
                atomicAdd(a.ovf + cell, 1);
                a.flags[b] = 1u;
            }
        }
    }
}

// One block per (kThreads correspondences, chunk of samples).
template <class KP>
__global__ __launch_bounds__(KP::kThreads, KP::kBlocksPerCU) void k_vote_keys(
    const float* __restrict__ x, const float* __restrict__ y, int64_t n, int G, float H, float gm,
    int J, int chunk, int ngroups, const float2* __restrict__ table, int nba, BinArgs a)
{
    __shared__ uint32_t stage[KP::kWaves][KP::kStageCap];
    __shared__ uint32_t s_cnt[kMaxBricksAll];
    __shared__ uint2 s_dst[kMaxBricksAll];
    __shared__ uint32_t s_scan[KP::kWaves];
    __shared__ uint32_t s_total;
    const int nb = nba * nba * nba;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int xs = (int)(blockIdx.x & (kSets - 1));
    const int cb = blockIdx.x / ngroups;
    const int gb = blockIdx.x - cb * ngroups;
    const int64_t i = (int64_t)gb * KP::kThreads + threadIdx.x;
    const int j0 = cb * chunk;
    const int j1 = min(J, j0 + chunk);
    for (int b = threadIdx.x; b < nb; b += KP::kThreads)
        s_cnt[b] = 0;
    __syncthreads();
    Quat u, v;
    const bool ok = load_circle(x, y, n, i, u, v);
    uint32_t* my_stage = stage[wave];
    const uint32_t wy = key_weight_y((uint32_t)nba), wz = key_weight_z((uint32_t)nba);
    uint32_t ends[kMaxBricksAll / KP::kThreads] = {};
    for (int js = j0; js < j1; js += KP::kWindow) {
        const int je = min(j1, js + KP::kWindow);
        for_samples<true>(u, v, table, js, je, H, gm, [&](const Cell& c, int j) {
            const uint32_t key = key_of(c, wy, wz);
            const int slot = (j - js) * kWave + lane;
            my_stage[slot] = ok ? key : kDropped;
            if (ok)
                atomicAdd(&s_cnt[key >> kKeyBrickShift], 1u);
        });
        keys_flush<KP>(stage, je - js, s_cnt, s_dst, s_scan, s_total, ends, wave, lane, nb, nba,
                       G, xs, a);
    }
}

// ----------------------------------------------------------- accumulate

// (w & 0xFFFF) << 2 in one instruction: the shift reads the low half-word
// (the compiler forms the high half-word's variant by itself, not this one).
__device__ __forceinline__ uint32_t low_half_x4(uint32_t w)
{
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "=v"(r)
        : "v"(2u), "v"(w));
    return r;
}

// kFmt: queue entries of narrow runs (spread local cell, length in byte 0),
// of wide runs (brick-local cell, length above bit 15) or keys (16-bit
// brick-local cells, one vote each).
template <int kLog, QueueFormat kFmt>
__global__ __launch_bounds__(Brick<kLog>::kThreads) void k_brick_accum(BinArgs a, int G, int nba, int K,
                                                                   int32_t* __restrict__ grid,
                                                                   uint64_t* __restrict__ partial)
{
    using Br = Brick<kLog>;
    constexpr int kEdge = Br::kEdge;
    constexpr int kBrickCells = Br::kCells;
    constexpr int kAccumThreads = Br::kThreads;
    constexpr int kAccumWaves = Br::kWaves;
    __shared__ uint32_t acc[kBrickCells];
    __shared__ uint64_t lists[kAccumWaves][kWave];
    __shared__ uint32_t s_floor, s_floor_top;
    const int nb = nba * nba * nba;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    uint4* acc4 = reinterpret_cast<uint4*>(acc);
    // A workgroup takes one brick per round of gridDim.x (persistent when the
    // launch has fewer workgroups than bricks); odd rounds run backwards, so
    // with bricks ordered heaviest first the workgroup with the heaviest brick
    // of one round gets the lightest of the next.
    const int items = a.batch ? (a.counts ? a.counts[1] : a.batch) * nb : nb;
    const int nwg = (int)gridDim.x;
    int round = 0;
    for (int base = 0; base < items; base += nwg, ++round) {
        const int item = base + ((round & 1) ? nwg - 1 - (int)blockIdx.x : (int)blockIdx.x);
        if (item >= items)
            continue;  // the whole workgroup: the last round is partial
        int inst, b;
        if (a.batch) {
            inst = item / nb;
            b = item - inst * nb;
        } else {
            inst = 0;
            b = (int)a.order[item];
        }
        const int set0 = 0, set1 = a.nsets;
        const int qoff = inst * nb;
        // this instance's grid and overflow grid (by its index in the batch)
        const int64_t gofs = (int64_t)(a.inst_of ? a.inst_of[inst] : inst) * G * G * G;
        const int bx = b % nba, by = (b / nba) % nba, bz = b / (nba * nba);

        // Without a grid to write, a brick that no run reached (nothing queued
        // in any set, nothing overflowed) holds only zero counts: its list is
        // empty and it needs no LDS pass.  Cells outside the chart's unit ball
        // are never voted, so about half of a large grid's bricks are empty.
        if (grid == nullptr) {
            uint32_t any = a.flags[qoff + b];
            for (int z = 0; z < a.nsets; ++z)
                any |= a.fill[(int64_t)z * a.qstride + qoff + b];
            if (any == 0u) {
                if (wave == 0)
                    partial[(int64_t)(qoff + b) * kWave + lane] = 0ull;
                continue;
            }
        }

        for (int k = threadIdx.x; k < kBrickCells / 4; k += kAccumThreads)
            acc4[k] = make_uint4(0u, 0u, 0u, 0u);
        if (threadIdx.x == 0) {
            s_floor = 0u;
            s_floor_top = 0xFFFFFFFFu;
        }
        __syncthreads();

        const uint32_t cap = a.cap[qoff + b];
        // The item's queue sets are read concurrently: the waves split into as
        // many groups as there are sets (at most one per wave), each group
        // streaming its sets in turn, so the latency of one set's first reads
        // overlaps the others'.  Software-pipelined queue reads: the next 8 KiB
        // per wave are in flight while the current ones are added into LDS.
        // Queues start on 64-entry boundaries and their capacity is a multiple
        // of 64, so 16-byte vector loads (4 runs or 8 keys) starting below the
        // fill count stay inside the queue.
        constexpr bool kKeys16 = kFmt == QueueFormat::kKeys;
        using Entry = typename std::conditional<kKeys16, uint16_t, uint32_t>::type;
        constexpr uint32_t kPerVec = 16 / sizeof(Entry);
        constexpr int kUnroll = 8;
        const int nset_here = set1 - set0;
        const int groups = min(kAccumWaves, nset_here);
        const int wpg = kAccumWaves / max(groups, 1);
        const int grp = wave / wpg;
        const uint32_t kStride = (uint32_t)wpg * kWave * kPerVec;
        for (int xs = set0 + grp; grp < groups && xs < set1; xs += groups) {
            const uint32_t cnt = min(a.fill[(int64_t)xs * a.qstride + qoff + b], cap);
            const Entry* q = reinterpret_cast<const Entry*>(a.pool) +
                             a.qbase[(int64_t)xs * a.qstride + qoff + b];
            if (cnt == 0)
                continue;
            // loads are unconditional (clamped to the queue's last vector) so the
            // compiler can keep the next batch in flight across the LDS atomics
            const uint32_t last = (cnt - 1u) & ~(kPerVec - 1u);
            uint4 cur[kUnroll], nxt[kUnroll];
            // Adds the entries of one vector whose first entry is number k
            // (every entry when `all`).  The LDS byte address is the cell index
            // times four, folded into the decode's weights and shifts.
            auto add_vec = [&](const uint4& v, uint32_t k, bool all) {
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    #pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if constexpr (kKeys16) {
                        // two keys per word; bit 15 of each is clear
                        if (all || k + 2 * i < cnt)
                            atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(acc) +
                                                                  low_half_x4(w[i])),
                                      1u);
                        if (all || k + 2 * i + 1 < cnt)
                            atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(acc) +
                                                                  ((w[i] >> 16) << 2)),
                                      1u);
                    } else {
                        uint32_t off, len;
                        const uint32_t e = w[i];
                        if constexpr (kFmt == QueueFormat::kNarrow) {
                            constexpr uint32_t kW4 = (4u << 8) | ((uint32_t)(4 * kEdge) << 16);
                            off = __builtin_amdgcn_udot4(e, kW4, (e >> 24) << (2 * kLog + 2), false);
                            len = e & 0xFFu;
                        } else {
                            off = (e << 2) & (0x7FFFu << 2);
                            len = e >> 15;
                        }
                        if (all || k + i < cnt)
                            atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(acc) + off),
                                      len);
                    }
                }
            };
            // kb: the wave's first entry of the batch (wave-uniform)
            uint32_t kb = (uint32_t)(wave - grp * wpg) * kWave * kPerVec;
            uint32_t k0 = kb + (uint32_t)lane * kPerVec;
            // non-temporal: each entry is read once, and streaming the queues
            // through L2 as ordinary lines took 12 % (one solve) to 25 % (the
            // key strategy's many small queues) longer
            auto load = [&](uint4 (&r)[kUnroll], uint32_t base) {
    #pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const v4u t = __builtin_nontemporal_load(
                        reinterpret_cast<const v4u*>(q + min(base + u * kStride, last)));
                    r[u] = make_uint4(t.x, t.y, t.z, t.w);
                }
            };
            load(cur, k0);
            while (kb < cnt) {
                const uint32_t kn = k0 + kStride * kUnroll;
                load(nxt, kn);
                if (cnt - kb >= (kUnroll - 1) * kStride + kWave * kPerVec) {
                    // every entry of the wave's batch is below cnt
    #pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        add_vec(cur[u], 0u, true);
                } else {
                    // entries past cnt add nothing
    #pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        add_vec(cur[u], k0 + u * kStride, false);
                }
    #pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    cur[u] = nxt[u];
                k0 = kn;
                kb += kStride * kUnroll;
            }
        }
        __syncthreads();

        // Pass 1: final counts (overflow runs added and written back to LDS), the
        // grid, and each lane's largest count.
        const bool overflowed = a.flags[qoff + b] != 0u;
        const bool vec = (G % 4) == 0;
        uint32_t lmax = 0;
        for (int c = threadIdx.x * 4; c < kBrickCells; c += kAccumThreads * 4) {
            const int lx = c & (kEdge - 1), ly = (c >> kLog) & (kEdge - 1), lz = c >> (2 * kLog);
            const int gx = bx * kEdge + lx, gy = by * kEdge + ly, gz = bz * kEdge + lz;
            uint32_t val[4] = {0u, 0u, 0u, 0u};
            const bool row = gy < G && gz < G;
            if (row) {
                const uint4 v4 = acc4[c >> 2];
                val[0] = v4.x; val[1] = v4.y; val[2] = v4.z; val[3] = v4.w;
                const int64_t g0 = ((int64_t)gz * G + gy) * G + gx;
                if (overflowed) {
    #pragma unroll
                    for (int s = 0; s < 4; ++s)
                        if (gx + s < G) {
                            val[s] += (uint32_t)a.ovf[gofs + g0 + s];
                            a.ovf[gofs + g0 + s] = 0;
                        }
                }
                if (overflowed)
                    acc4[c >> 2] = make_uint4(val[0], val[1], val[2], val[3]);
                if (grid == nullptr) {
                    // batch without grids: only the brick's list leaves the CU
                } else if (vec && gx + 3 < G) {
                    *reinterpret_cast<int4*>(grid + gofs + g0) =
                        make_int4((int)val[0], (int)val[1], (int)val[2], (int)val[3]);
                } else {
    #pragma unroll
                    for (int s = 0; s < 4; ++s)
                        if (gx + s < G)
                            grid[gofs + g0 + s] = (int32_t)val[s];
                }
            }
            // cells past the grid's edge hold 0 and cannot raise the maximum
            lmax = max(lmax, max(max(val[0], val[1]), max(val[2], val[3])));
        }
        // A floor for the top K.  Lane maxima are counts of distinct cells, so
        // the brick's K-th largest count is at least (1) the K-th largest lane
        // maximum of any one wave, and (2) the smallest, over the waves, of
        // each wave's ceil(K / waves)-th largest lane maximum (every wave has
        // that many at or above it, K in all).  In a dense brick (2) is far
        // higher: it leaves pass 2 a few cells instead of most of them.
        // Cells below the floor cannot be among the brick's K best and skip
        // the list.
        const uint64_t srt = wave_sort_desc((uint64_t)lmax, lane);
        const uint32_t kth = (uint32_t)lane_u64(srt, K - 1);
        const uint32_t top = (uint32_t)lane_u64(srt, (K + kAccumWaves - 1) / kAccumWaves - 1);
        if (lane == 0) {
            atomicMax(&s_floor, kth);
            atomicMin(&s_floor_top, top);
        }
        __syncthreads();
        const uint32_t floor_k = max(max(s_floor, s_floor_top), 1u);

        // Pass 2: the sorted list of the brick's best cells at or above the floor.
        uint64_t list = 0;
        for (int c = threadIdx.x * 4; c < kBrickCells; c += kAccumThreads * 4) {
            const int lx = c & (kEdge - 1), ly = (c >> kLog) & (kEdge - 1), lz = c >> (2 * kLog);
            const int gx = bx * kEdge + lx, gy = by * kEdge + ly, gz = bz * kEdge + lz;
            const bool row = gy < G && gz < G;
            const uint4 v4 = acc4[c >> 2];
            const uint32_t val[4] = {v4.x, v4.y, v4.z, v4.w};
            const bool hit = row && max(max(val[0], val[1]), max(val[2], val[3])) >= floor_k;
            if (__ballot(hit) == 0)  // the common case: no cell of the wave's 256 qualifies
                continue;
            const uint32_t idx0 = (uint32_t)(((int64_t)gz * G + gy) * G + gx);
    #pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bool in = row && gx + s < G && val[s] >= floor_k;
                list = wave_insert_top(list, in ? cell_key(val[s], idx0 + s) : 0ull, lane, K);
            }
        }
        list = block_merge<kAccumWaves>(list, lists, wave, lane);
        if (wave == 0)
            partial[(int64_t)(qoff + b) * kWave + lane] = list;
        __syncthreads();  // the LDS is reused by the next brick
    }
}

// ------------------------------------------------------------- launchers

int brick_axis(int G, int edge_log2) { return (G + (1 << edge_log2) - 1) >> edge_log2; }

namespace {

constexpr int kMaxDevices = 64;

// Workgroups of the persistent accumulation: as many as the device holds at
// once (CUs x resident workgroups per CU, measured once per device and edge),
// at most one per brick.
int accum_blocks(int edge_log2, int items)
{
    static std::atomic<int> cached[2][kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return items;
    std::atomic<int>& slot = cached[edge_log2 == 5 ? 1 : 0][dev];
    int v = slot.load(std::memory_order_relaxed);
    if (v <= 0) {
        int cus = 0, occ = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return items;
        const hipError_t e =
            edge_log2 == 5
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_brick_accum<5, QueueFormat::kNarrow>,
                                                               Brick<5>::kThreads, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_brick_accum<4, QueueFormat::kNarrow>,
                                                               Brick<4>::kThreads, 0);
        if (e != hipSuccess || cus < 1 || occ < 1)
            return items;
        v = cus * occ;
        slot.store(v, std::memory_order_relaxed);
    }
    return std::max(1, std::min(items, v));
}

// Compute units of the current device (cached per device).
int device_cus()
{
    static std::atomic<int> cached[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return 256;
    int v = cached[dev].load(std::memory_order_relaxed);
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
            return 256;
        cached[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Samples per vote workgroup.  A launch of ngroups x n workgroups runs
// `resident` of them at a time; each costs its samples plus about
// kChunkCost sample-equivalents (circle set-up, its last partial flush), and
// the last ones to start leave the GPU partly idle for about half a
// workgroup: n = sqrt(J resident / (2 ngroups kChunkCost)) balances the two.
// Workgroups start in chunk order, so the first n - 1 chunks are equal and
// the last about a quarter of their length: the launch's last, partial round
// is then made of short workgroups.  Chunks are whole multiples of `unit`
// samples.  (Measured on one solve at N = 1e6, G = 256, J = 2048: one chunk
// 2.33 ms, five equal 2.14, four of 480 and one of 128 samples 2.09; at
// N = 1e5, G = 128, J = 1024: five of 240 samples 0.171 ms, eight equal
// 0.157, ten of 96 and one of 64 0.141.)
int vote_chunk(int J, int64_t ngroups, int64_t resident, int unit)
{
    constexpr double kChunkCost = 16.0;
    const double best = std::sqrt((double)J * (double)resident / (2.0 * (double)ngroups * kChunkCost));
    const int64_t units = (J + unit - 1) / unit;
    const int64_t n = std::min<int64_t>(std::max<int64_t>(1, std::llround(best)), units);
    if (n <= 1)
        return (int)(units * unit);
    const double full = ((double)J - (double)J / (4.0 * (double)n)) / (double)(n - 1);
    return (int)(std::max<int64_t>(1, (int64_t)(full / (double)unit)) * unit);
}

}  // namespace

int solve_edge_log2(int G) { return G <= 128 ? 4 : 5; }

hipError_t launch_bin_prepare(const float* x, const float* y, int64_t n, int G, int J,
                              int edge_log2, const float2* table, const BinArgs& a, hipStream_t s,
                              bool keys)
{
    const bool wide = G > kNarrowGrid;
    if ((edge_log2 != 4 && edge_log2 != 5) || (edge_log2 == 4 && (wide || keys)))
        return hipErrorInvalidValue;
    const int nba = brick_axis(G, edge_log2);
    const int nb = nba * nba * nba;
    if (G > kMaxBrickGrid || nb > ((wide || keys) ? kMaxBricksAll : kMaxBricks))
        return hipErrorInvalidValue;
    const float H = (float)G * 0.5f;
    const float gm = (float)G - 0.5f;
    const int stride = estimate_stride(n, keys);
    if (n > 0) {
        const int64_t nsamp = (n + stride - 1) / stride;
        const int64_t ngroups = (nsamp + kWave - 1) / kWave;
        // chunks of whole table rows (8 samples) for about 4096 waves
        const int64_t rows = (J + 7) / 8;
        const int64_t want = (4096 + ngroups - 1) / ngroups;
        const int64_t nch = std::min<int64_t>(std::max<int64_t>(want, 1), rows);
        const int chunk = (int)(((rows + nch - 1) / nch) * 8);
        const int64_t nchunks = (J + chunk - 1) / chunk;
        const int64_t nwaves = ngroups * nchunks;
        if (nwaves > (int64_t)INT32_MAX - 4)
            return hipErrorInvalidValue;
        const dim3 grid((unsigned)((nwaves + 3) / 4));
        if (keys)
            hipLaunchKernelGGL((k_bin_estimate<5, true, true>), grid, dim3(256), 0, s, x, y, n, H,
                               gm, J, table, nba, chunk, (int)ngroups, (int)nwaves, stride, a.est);
        else if (wide)
            hipLaunchKernelGGL((k_bin_estimate<5, true, false>), grid, dim3(256), 0, s, x, y, n, H,
                               gm, J, table, nba, chunk, (int)ngroups, (int)nwaves, stride, a.est);
        else if (edge_log2 == 5)
            hipLaunchKernelGGL((k_bin_estimate<5, false, false>), grid, dim3(256), 0, s, x, y, n, H,
                               gm, J, table, nba, chunk, (int)ngroups, (int)nwaves, stride, a.est);
        else
            hipLaunchKernelGGL((k_bin_estimate<4, false, false>), grid, dim3(256), 0, s, x, y, n, H,
                               gm, J, table, nba, chunk, (int)ngroups, (int)nwaves, stride, a.est);
        if (hipError_t e = hipGetLastError(); e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_bin_plan, dim3(1), dim3(kPlanThreads), 0, s, a, nb, stride);
    return hipGetLastError();
}

hipError_t launch_key_vote(const float* x, const float* y, int64_t n, int G, int J,
                           const float2* table, const BinArgs& a, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int nba = brick_axis(G, 5);
    if (G > kMaxBrickGrid || nba * nba * nba > kMaxBricksAll || a.units || a.nsets != kSets)
        return hipErrorInvalidValue;
    const int64_t ngroups = (n + Keys::kThreads - 1) / Keys::kThreads;
    // J split into whole flush windows (vote_chunk)
    const int chunk = vote_chunk(J, ngroups, (int64_t)Keys::kBlocksPerCU * device_cus(), Keys::kWindow);
    const int64_t nchunks = (J + chunk - 1) / chunk;
    const int64_t blocks = ngroups * nchunks;
    if (blocks > INT32_MAX)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_vote_keys<Keys>), dim3((unsigned)blocks), dim3(Keys::kThreads), 0, s, x, y,
                       n, G, (float)G * 0.5f, (float)G - 0.5f, J, chunk, (int)ngroups, table, nba, a);
    return hipGetLastError();
}

hipError_t launch_bin_vote(const float* x, const float* y, int64_t n, int G, int J, int edge_log2,
                           const float2* table, const BinArgs& a, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const bool wide = G > kNarrowGrid;
    if ((edge_log2 != 4 && edge_log2 != 5) || (edge_log2 == 4 && wide))
        return hipErrorInvalidValue;
    const int threads = wide ? Pack<true>::kThreads : Pack<false>::kThreads;
    const int64_t ngroups = (n + threads - 1) / threads;
    // J split into whole table rows of 8 samples (vote_chunk); runs are cut
    // at chunk starts and every kSplit samples after
    const int chunk = vote_chunk(
        J, ngroups, (int64_t)(wide ? Pack<true>::kBlocksPerCU : Pack<false>::kBlocksPerCU) * device_cus(), 8);
    const int64_t nchunks = (J + chunk - 1) / chunk;
    const int64_t blocks = ngroups * nchunks;
    if (blocks > INT32_MAX || G > kMaxBrickGrid)
        return hipErrorInvalidValue;
    if (wide)
        hipLaunchKernelGGL((k_vote_bin<5, true>), dim3((unsigned)blocks), dim3(threads), 0, s, x,
                           y, n, G, (float)G * 0.5f, (float)G - 0.5f, J, chunk, (int)ngroups, table,
                           brick_axis(G, 5), a);
    else if (edge_log2 == 5)
        hipLaunchKernelGGL((k_vote_bin<5, false>), dim3((unsigned)blocks), dim3(threads), 0, s, x,
                           y, n, G, (float)G * 0.5f, (float)G - 0.5f, J, chunk, (int)ngroups, table,
                           brick_axis(G, 5), a);
    else
        hipLaunchKernelGGL((k_vote_bin<4, false>), dim3((unsigned)blocks), dim3(threads), 0, s, x,
                           y, n, G, (float)G * 0.5f, (float)G - 0.5f, J, chunk, (int)ngroups, table,
                           brick_axis(G, 4), a);
    return hipGetLastError();
}

hipError_t launch_brick_accum(int G, int K, int edge_log2, QueueFormat fmt, int32_t* grid,
                              uint64_t* partial, const BinArgs& a, hipStream_t s)
{
    if ((edge_log2 != 4 && edge_log2 != 5) || (edge_log2 == 4 && fmt != QueueFormat::kNarrow))
        return hipErrorInvalidValue;
    const int nba = brick_axis(G, edge_log2);
    const int nb = nba * nba * nba;
    if (G > kMaxBrickGrid || nb > kMaxBricksAll)
        return hipErrorInvalidValue;
    if (K < 1 || K > kWave)
        return hipErrorInvalidValue;
    // batches of 32^3 bricks: persistent workgroups (measured 5 % faster over
    // 32 768 bricks); 16^3 bricks (many small workgroups per CU) and one solve:
    // a workgroup per brick, which the hardware hands out in order (the plan's
    // heaviest first) as CUs free up (persistent was slower there)
    // (a batch planned on the device, of either edge, is launched persistent
    // for its upper bound of bricks)
    const int blocks = (a.batch && (edge_log2 == 5 || a.counts)) ? accum_blocks(edge_log2, a.batch * nb)
                                                                 : (a.batch ? a.batch * nb : nb);
    if (edge_log2 == 4)
        hipLaunchKernelGGL((k_brick_accum<4, QueueFormat::kNarrow>), dim3(blocks),
                           dim3(Brick<4>::kThreads), 0, s, a, G, nba, K, grid, partial);
    else if (fmt == QueueFormat::kNarrow)
        hipLaunchKernelGGL((k_brick_accum<5, QueueFormat::kNarrow>), dim3(blocks),
                           dim3(Brick<5>::kThreads), 0, s, a, G, nba, K, grid, partial);
    else if (fmt == QueueFormat::kWide)
        hipLaunchKernelGGL((k_brick_accum<5, QueueFormat::kWide>), dim3(blocks),
                           dim3(Brick<5>::kThreads), 0, s, a, G, nba, K, grid, partial);
    else
        hipLaunchKernelGGL((k_brick_accum<5, QueueFormat::kKeys>), dim3(blocks),
                           dim3(Brick<5>::kThreads), 0, s, a, G, nba, K, grid, partial);
    return hipGetLastError();
}

hipError_t launch_bin_vote_batch(const float* x, const float* y, int64_t n, int G, int J,
                                 int edge_log2, const float2* table, const BinArgs& a, int nunits,
                                 hipStream_t s)
{
    if (nunits <= 0)
        return hipSuccess;
    if (G > kMaxBrickGrid || !a.units || (edge_log2 != 4 && edge_log2 != 5))
        return hipErrorInvalidValue;
    const int nba = brick_axis(G, edge_log2);
    if (nba * nba * nba > kMaxBricks)
        return hipErrorInvalidValue;
    if (edge_log2 == 5)
        hipLaunchKernelGGL((k_vote_bin<5, false>), dim3((unsigned)nunits), dim3(Pack<false>::kThreads), 0, s, x,
                           y, n, G, (float)G * 0.5f, (float)G - 0.5f, J, J, 1, table, nba, a);
    else
        hipLaunchKernelGGL((k_vote_bin<4, false>), dim3((unsigned)nunits), dim3(Pack<false>::kThreads), 0, s, x,
                           y, n, G, (float)G * 0.5f, (float)G - 0.5f, J, J, 1, table, nba, a);
    return hipGetLastError();
}

}  // namespace rv
