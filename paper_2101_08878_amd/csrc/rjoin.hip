// Radix join: the per-partition inner join (arXiv 2101.08878, Section V-B
// "cuDF Merge": every worker merges the frames it received) with every table
// held in LDS.
//
// Both sides arrive split into sub-buckets (partition p, top hash bits q), so
// that a sub-bucket's build rows fit one workgroup's LDS.  A workgroup takes
// sub-buckets in order from a ticket counter; for each it
//   1. loads the build rows into LDS: key, payload, and a chain link; bucket
//      heads hold the last row inserted per bucket (LDS atomic exchange), so
//      equal keys share a chain and repeated keys need nothing special;
//   2. counts the output rows of all its probe rows (walking each row's
//      chain) and takes the output row of its first one (output placement,
//      below);
//   3. writes (key, left payload, right payload) rows.  When the probe rows
//      fit one batch (4096 rows) they stay in registers between 2 and 3;
//      otherwise they are read and looked up again.
// Sub-buckets are numbered partition-major, and partition p's output is the
// contiguous range [out_off[p], out_off[p+1]).  Global memory is only
// streamed: the random accesses of the join all hit LDS.  The partition
// already sent each key to its sub-bucket by fmix64, so inside a sub-bucket a
// key's chain is chosen by a one-multiply hash of the key itself and keys are
// compared directly: fmix64 (six 32-bit multiplies, quarter-rate
// instructions) is not computed again here.
//
// Latency hiding: two workgroups per CU, one running while the other waits
// on the dependent steps of its sub-bucket; inside a sub-bucket the loads
// are issued in the order they are needed (join_one_batch), and the hash
// chains of a thread's probe rows are walked four at a time without
// branches, so that their LDS reads are in flight together.
#include <algorithm>

#include "mdx.h"
#include "mdx_internal.hpp"

namespace mdx {
namespace {

constexpr int kJoinWaves = kJoinThreads / kWave;
constexpr int kBuildBatch = 8;  // build rows per thread loaded together
constexpr int kCells = kJoinRows * kJoinWaves;  // (row step, wave) partial sums
constexpr int kCellsPerLane = kCells / kWave;
static_assert(kCells % kWave == 0, "one wave scans the partial sums");

// A table of geometry G (G::cap build rows, G::heads chain heads).  Chains
// end at the sentinel row `sent` (one slot past the table), whose link
// points to itself.
template <class G>
struct Tab {
    static constexpr uint32_t sent = G::cap;
    static constexpr int log_heads = __builtin_ctz(G::heads);
    static_assert(G::cap <= 0xffff, "chain links are 16-bit");
    static_assert((G::heads & (G::heads - 1)) == 0, "power-of-two heads");
    static_assert(kBuildBatch * kJoinThreads >= G::cap, "one load batch per table");
    static_assert(kJoinRows % G::walk == 0, "walk groups tile the thread's rows");
};

// Chain of a key inside its sub-bucket: multiplicative (Fibonacci) hashing
// of the key's two 32-bit halves folded together.
template <class G>
__device__ __forceinline__ uint32_t bucket_of(int64_t key)
{
    const uint32_t x = (uint32_t)key ^ (uint32_t)((uint64_t)key >> 32);
    return (x * 0x9E3779B1u) >> (32 - Tab<G>::log_heads);
}

// Values every lane of the workgroup holds alike, in scalar registers.
__device__ __forceinline__ int64_t uniform(int64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ---- output placement ------------------------------------------------------
// Partition p's output rows form one range, [base(p), base(p+1)); the order
// of its sub-buckets' rows inside that range is free (row order inside a
// partition is implementation-defined).  Two ways to place them:
//  - by sub-bucket: a chained scan over all sub-buckets in ticket order
//    (pst[s] its status, part[s] its first output row).  A sub-bucket
//    waits until every sub-bucket ticketed before it has been counted.
//  - by partition: a sub-bucket takes its rows from its partition's cursor
//    part[p] with one atomic add (the low kDoneBits count the sub-buckets
//    counted, the bits above the rows taken), and base(p) is the exclusive
//    prefix of the partition totals, a chained scan over the P entries of
//    pst: the last sub-bucket of p to be counted publishes p's total.  A
//    sub-bucket then waits only while an earlier partition still has
//    sub-buckets being counted.  The sub-buckets of earlier partitions were
//    all ticketed before this one, to running workgroups, so the wait ends.
// By partition pays when partitions hold many more sub-buckets than there
// are workgroups: then few sub-buckets wait at all (1E8 x 1E8 at P = 1:
// 13.7 instead of 18.4 us per sub-bucket and workgroup).  With partitions
// of ~2 workgroups' worth (P = 32), half the sub-buckets in flight wait for
// the partition before and are all released at once when it completes, and
// their output writes then contend (21 us per sub-bucket): by sub-bucket.
struct Place {
    uint64_t *part;   // by partition: [P] rows taken << kDoneBits | counted;
                      // by sub-bucket: [S] first output row of each
    uint64_t *pst;    // [P] or [S]: chained-scan status
    int32_t qbits;    // 2^qbits sub-buckets per partition (qbits < kDoneBits)
    int32_t by_part;  // 1: by partition, 0: by sub-bucket
};
// A merge has at most 2^22 sub-buckets, so the count of a partition's never
// carries into its rows; the rows taken are kept modulo 2^41 (a carry out
// of them is lost), and a partition reaching 2^41 output rows (far beyond
// any output buffer) is reported as an output overflow.
constexpr int kDoneBits = 23;
constexpr uint64_t kDoneMask = (1ull << kDoneBits) - 1;
constexpr uint64_t kRowsLimit = 1ull << (64 - kDoneBits);

// Wave 0 of a workgroup: the output row of sub-bucket s's first row, for its
// `total` rows.  (cp, cb): the workgroup's last partition and that
// partition's base, kept across sub-buckets (cp = -1: none yet).
__device__ inline int64_t place_rows(const Place &pl, int64_t s, int64_t total, int &cp,
                                     int64_t &cb, int lane, int32_t *status)
{
    if (!pl.by_part) {
        const int64_t ex = lookback(pl.pst, s, total, lane, status);
        if (lane == 0)
            pl.part[s] = (uint64_t)ex;
        return ex;
    }
    const int p = (int)(s >> pl.qbits);
    uint64_t old = 0;
    if (lane == 0)
        old = atomicAdd((unsigned long long *)(pl.part + p), ((uint64_t)total << kDoneBits) + 1);
    old = __shfl(old, 0, kWave);
    const uint64_t before = old >> kDoneBits;  // rows of p taken before these
    if (lane == 0 && ((uint64_t)total >= kRowsLimit || before + (uint64_t)total >= kRowsLimit))
        or_status(status, MDX_DEV_OUTPUT_OVERFLOW);
    if (lane == 0 && (old & kDoneMask) + 1 == (1ull << pl.qbits))
        st_agent(pl.pst + p, kFlagAgg | (before + (uint64_t)total));
    if (p != cp) {
        bool ok;
        cb = prefix_before(pl.pst, p, lane, status, &ok);
        // p - 1's inclusive prefix is base(p): later look-backs stop there
        if (ok && p > 0 && lane == 0)
            st_agent(pl.pst + p - 1, kFlagIncl | (uint64_t)cb);
        cp = p;
    }
    return cb + (int64_t)before;
}

// chunked: oversized build sub-buckets are joined in chunks (the LDS-fit
// flag stays 1).
__global__ __launch_bounds__(kBlock) void rj_plan(const int64_t *__restrict__ subL, int64_t S,
                                                  RJoinWs w, int chunked)
{
    int over = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < S; s += stride) {
        w.status[s] = 0;
        w.tile_base[s] = 0;
        over |= (subL[s + 1] - subL[s]) > kJoinCap;
    }
    if (over && !chunked)
        *w.use = 0;  // rj_plan_init set it to 1 before this kernel
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *w.ticket = 0;
}

__global__ void rj_plan_init(RJoinWs w)
{
    *w.use = 1;
}

// One block for the whole plan when there are few sub-buckets: the flag is
// decided by a block-wide OR, so it needs no earlier kernel to set it.
constexpr int kPlanOnePerThread = 8;

__global__ __launch_bounds__(kBlock) void rj_plan_one(const int64_t *__restrict__ subL, int64_t S,
                                                      RJoinWs w, int chunked)
{
    // Every thread's loads are issued together: indices past S are clamped
    // to S - 1 (S >= 1) and their results ignored, so no load sits behind a
    // branch.
    int64_t a[kPlanOnePerThread], b[kPlanOnePerThread];
#pragma unroll
    for (int k = 0; k < kPlanOnePerThread; ++k) {
        const int64_t s = threadIdx.x + (int64_t)k * kBlock;
        const int64_t c = s < S ? s : S - 1;
        a[k] = subL[c];
        b[k] = subL[c + 1];
    }
    int over = 0;
#pragma unroll
    for (int k = 0; k < kPlanOnePerThread; ++k) {
        const int64_t s = threadIdx.x + (int64_t)k * kBlock;
        over |= s < S && b[k] - a[k] > kJoinCap;
        if (s < S) {
            w.status[s] = 0;
            w.tile_base[s] = 0;
        }
    }
    over = __syncthreads_or(over);
    if (threadIdx.x == 0) {
        *w.use = over && !chunked ? 0 : 1;
        *w.ticket = 0;
    }
}

// Sub-buckets up to which rj_plan_one runs.
constexpr int64_t kPlanOneMax = (int64_t)kBlock * kPlanOnePerThread;

// This thread's rows of the batch starting at rb (the same on every lane),
// up to re (rb < re): rb + j kJoinThreads + tid.  Rows past re load the
// batch's last row instead (no branch per load) and are ignored by the
// callers, which check r < re.
template <typename K>
__device__ __forceinline__ void load_batch(const K *__restrict__ rk, const int64_t *__restrict__ rv,
                                           int64_t rb, int64_t re, K *kk, int64_t *vv)
{
    const K *kb = rk + rb;
    const int64_t *vb = rv + rb;
    const int64_t left = re - rb;
    const uint32_t last = (uint32_t)((left < kJoinBatch ? left : kJoinBatch) - 1);
#pragma unroll
    for (int j = 0; j < kJoinRows; ++j) {
        uint32_t r = (uint32_t)(j * kJoinThreads) + threadIdx.x;
        r = r < last ? r : last;
        kk[j] = __builtin_nontemporal_load(kb + r);
        vv[j] = __builtin_nontemporal_load(vb + r);
    }
}

// Per row: the number of matches (high 16 bits; at most G::cap) and the
// first matching build row in chain order (low 16 bits; meaningful when the
// count is not 0).  The chains of G::walk rows are walked together without
// branches: a finished chain sits on the sentinel row, whose link points to
// itself, so every step issues all G::walk rows' LDS reads at once.
template <class G, typename K>
__device__ __forceinline__ void match_batch(int64_t rb, int64_t re, bool any, const int64_t *tkey,
                                            const uint16_t *tn, const uint32_t *head, const K *kk,
                                            uint32_t *mf)
{
    constexpr uint32_t kSent = Tab<G>::sent;
    constexpr int kWalk = G::walk;
    const int64_t left = re - rb;
    const uint32_t n = any ? (uint32_t)(left < kJoinBatch ? left : kJoinBatch) : 0u;
#pragma unroll
    for (int g = 0; g < kJoinRows; g += kWalk) {
        int64_t h[kWalk];
        uint32_t e[kWalk];
        bool live = false;
#pragma unroll
        for (int i = 0; i < kWalk; ++i) {
            const int j = g + i;
            const uint32_t r = (uint32_t)(j * kJoinThreads) + threadIdx.x;
            mf[j] = 0;
            h[i] = (int64_t)kk[j];
            e[i] = r < n ? head[bucket_of<G>(h[i])] : kSent;
            live |= e[i] != kSent;
        }
        while (ballot(live)) {
            int64_t x[kWalk];
            uint32_t nx[kWalk];
#pragma unroll
            for (int i = 0; i < kWalk; ++i) {
                x[i] = tkey[e[i]];
                nx[i] = tn[e[i]];
            }
            live = false;
#pragma unroll
            for (int i = 0; i < kWalk; ++i) {
                const int j = g + i;
                if (x[i] == h[i] && e[i] != kSent)
                    mf[j] = mf[j] == 0 ? ((1u << 16) | e[i]) : mf[j] + (1u << 16);
                e[i] = nx[i];
                live |= e[i] != kSent;
            }
        }
    }
}

// Per-(row step, wave) sums of the match counts into cw (row order =
// step-major).  When no row of the step matches twice, the sum is a
// population count.
__device__ __forceinline__ void cell_sums(const uint32_t *mf, int64_t *cw, int lane, int wv)
{
#pragma unroll
    for (int j = 0; j < kJoinRows; ++j) {
        const uint32_t cnt = mf[j] >> 16;
        const uint64_t one = ballot(cnt == 1), many = ballot(cnt > 1);
        const int64_t s = many ? wave_sum((int64_t)cnt) : (int64_t)__popcll(one);
        if (lane == 0)
            cw[j * kJoinWaves + wv] = s;
    }
}

// Wave 0: total of the cells.
__device__ __forceinline__ int64_t cell_total(const int64_t *cw, int lane)
{
    int64_t loc = 0;
#pragma unroll
    for (int i = 0; i < kCellsPerLane; ++i)
        loc += cw[lane * kCellsPerLane + i];
    return wave_sum(loc);
}

// Wave 0: cw := exclusive prefix of cw (step-major), returns the total.
__device__ __forceinline__ int64_t cell_scan(int64_t *cw, int lane)
{
    int64_t v[kCellsPerLane], loc = 0;
#pragma unroll
    for (int i = 0; i < kCellsPerLane; ++i) {
        v[i] = cw[lane * kCellsPerLane + i];
        loc += v[i];
    }
    const int64_t inc = wave_incl_scan(loc, lane);
    int64_t run = inc - loc;
#pragma unroll
    for (int i = 0; i < kCellsPerLane; ++i) {
        cw[lane * kCellsPerLane + i] = run;
        run += v[i];
    }
    return __shfl(inc, kWave - 1, kWave);
}

// Write the output rows of the batch held in registers; base = output row of
// the batch's first match; cw holds the exclusive cell prefixes.
template <class G, typename K>
__device__ __forceinline__ void emit_batch(const K *kk, const int64_t *vv, const uint32_t *mf,
                                           const int64_t *cw, int64_t base, const int64_t *tkey,
                                           const int64_t *tp, const uint16_t *tn, K *out_key,
                                           int64_t *out_l, int64_t *out_r, int lane, int wv)
{
    constexpr uint32_t kSent = Tab<G>::sent;
#pragma unroll
    for (int j = 0; j < kJoinRows; ++j) {
        const uint32_t cnt = mf[j] >> 16, fst = mf[j] & 0xffffu;
        const uint64_t one = ballot(cnt == 1), many = ballot(cnt > 1);
        if (!(one | many))
            continue;
        const int64_t before =
            many ? wave_incl_scan((int64_t)cnt, lane) - (int64_t)cnt : (int64_t)mbcnt(one);
        // the wave's first output row of this step: a scalar base; lanes add
        // a 32-bit offset (a step of a wave has at most 64 G::cap rows)
        const int64_t wb = uniform(base + cw[j * kJoinWaves + wv]);
        K *ok = out_key + wb;
        int64_t *ol = out_l + wb, *orr = out_r + wb;
        uint32_t at = (uint32_t)before;
        if (cnt == 1) {
            ok[at] = kk[j];
            ol[at] = tp[fst];
            orr[at] = vv[j];
        } else if (cnt > 1) {
            const int64_t h = (int64_t)kk[j];
            for (uint32_t e = fst; e != kSent; e = tn[e]) {
                if (tkey[e] == h) {
                    ok[at] = kk[j];
                    ol[at] = tp[e];
                    orr[at] = vv[j];
                    ++at;
                }
            }
        }
    }
}

// Insert build rows [b0, b0 + n) (0 < n <= G::cap) into the LDS table,
// kBuildBatch rows per thread at a time.  Rows past n load the last row (no
// branch per load) and are not inserted.
template <class G, typename K>
__device__ __forceinline__ void build_table(const K *__restrict__ lk,
                                            const int64_t *__restrict__ lv, int64_t b0, int64_t n,
                                            int64_t *tkey, int64_t *tp, uint16_t *tn,
                                            uint32_t *head)
{
    const int tid = threadIdx.x;
    for (int i = tid; i < G::heads; i += kJoinThreads)
        head[i] = Tab<G>::sent;
    __syncthreads();
    const K *kb = lk + b0;
    const int64_t *vb = lv + b0;
    const uint32_t last = (uint32_t)n - 1;
    for (int base = 0; base < (int)n; base += kBuildBatch * kJoinThreads) {
        K bk[kBuildBatch];
        int64_t bv[kBuildBatch];
#pragma unroll
        for (int j = 0; j < kBuildBatch; ++j) {
            uint32_t i = (uint32_t)(base + j * kJoinThreads) + tid;
            i = i < last ? i : last;
            bk[j] = __builtin_nontemporal_load(kb + i);
            bv[j] = __builtin_nontemporal_load(vb + i);
        }
#pragma unroll
        for (int j = 0; j < kBuildBatch; ++j) {
            const int i = base + j * kJoinThreads + tid;
            if (i < n) {
                const int64_t k = (int64_t)bk[j];
                tkey[i] = k;
                tp[i] = bv[j];
                tn[i] = (uint16_t)atomicExch(&head[bucket_of<G>(k)], (uint32_t)i);
            }
        }
    }
    __syncthreads();
}

// The LDS of a join workgroup.
struct JoinLds {
    int64_t *tkey;  // [G::cap + 1] key of build row i
    int64_t *tp;    // [G::cap] payload of build row i
    uint16_t *tn;   // [G::cap + 1] next row in i's chain
    uint32_t *head; // [G::heads] last row inserted per bucket
    int64_t *cw;    // [kCells]
    int64_t *s_excl, *s_total;
};

// The common sub-bucket: its build rows fit one table and its probe rows one
// batch (0 < nb <= G::cap, 0 < eR - bR <= kJoinBatch).  A wave's loads
// complete in the order they were issued, and waiting for one waits for all
// issued before it; so they are issued in the order they are needed, with
// no branch around any of them (so that the compiler counts them exactly):
// the build rows (the inserts wait for these alone), the probe keys (the
// match), then, once the table is built, the probe payloads (needed only to
// write the output, so they arrive during the count and the chained scan).
template <class G, typename K>
__device__ __forceinline__ void join_one_batch(const K *__restrict__ lk,
                                               const int64_t *__restrict__ lv, int64_t bL,
                                               int64_t nb, const K *__restrict__ rk,
                                               const int64_t *__restrict__ rv, int64_t bR,
                                               int64_t eR, const Place &pl, int64_t s, int &cp,
                                               int64_t &cb, const ProbeOut &o, int32_t *status,
                                               const JoinLds &L)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const uint32_t blast = (uint32_t)nb - 1, plast = (uint32_t)(eR - bR) - 1;
    K bk[kBuildBatch];
    int64_t bv[kBuildBatch];
#pragma unroll
    for (int j = 0; j < kBuildBatch; ++j) {
        const uint32_t i = (uint32_t)(j * kJoinThreads + tid);
        bk[j] = __builtin_nontemporal_load(lk + bL + (i < blast ? i : blast));
    }
#pragma unroll
    for (int j = 0; j < kBuildBatch; ++j) {
        const uint32_t i = (uint32_t)(j * kJoinThreads + tid);
        bv[j] = __builtin_nontemporal_load(lv + bL + (i < blast ? i : blast));
    }
    K kk[kJoinRows];
#pragma unroll
    for (int j = 0; j < kJoinRows; ++j) {
        const uint32_t r = (uint32_t)(j * kJoinThreads + tid);
        kk[j] = __builtin_nontemporal_load(rk + bR + (r < plast ? r : plast));
    }
    for (int i = tid; i < G::heads; i += kJoinThreads)
        L.head[i] = Tab<G>::sent;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBuildBatch; ++j) {
        const int i = j * kJoinThreads + tid;
        if (i < nb) {
            const int64_t k = (int64_t)bk[j];
            L.tkey[i] = k;
            L.tp[i] = bv[j];
            L.tn[i] = (uint16_t)atomicExch(&L.head[bucket_of<G>(k)], (uint32_t)i);
        }
    }
    __syncthreads();
    int64_t vv[kJoinRows];
#pragma unroll
    for (int j = 0; j < kJoinRows; ++j) {
        const uint32_t r = (uint32_t)(j * kJoinThreads + tid);
        vv[j] = __builtin_nontemporal_load(rv + bR + (r < plast ? r : plast));
    }

    uint32_t mf[kJoinRows];
    match_batch<G>(bR, eR, true, L.tkey, L.tn, L.head, kk, mf);
    cell_sums(mf, L.cw, lane, wv);
    __syncthreads();
    if (wv == 0) {
        const int64_t total = cell_scan(L.cw, lane);
        const int64_t ex = place_rows(pl, s, total, cp, cb, lane, status);
        if (lane == 0) {
            *L.s_excl = ex;
            *L.s_total = total;
        }
    }
    __syncthreads();
    const int64_t E = *L.s_excl, total = *L.s_total;
    if (E + total > o.cap) {
        if (tid == 0 && total > 0)
            or_status(status, MDX_DEV_OUTPUT_OVERFLOW);
    } else if (total > 0) {
        emit_batch<G>(kk, vv, mf, L.cw, E, L.tkey, L.tp, L.tn, (K *)o.key, o.lpay, o.rpay, lane,
                      wv);
    }
}

// Sub-bucket s of one merge: build rows [bL, bL + nb), probe rows [bR, eR).
// Counts its output rows, takes them from its partition (place_rows), then
// writes them.  With CHUNKED,
// a build side larger than the table is joined one table-sized chunk at a
// time (every chunk against every probe row: each pair of rows meets once);
// otherwise nb <= G::cap.
template <class G, typename K, bool CHUNKED>
__device__ __forceinline__ void join_sub_bucket(const K *__restrict__ lk,
                                                const int64_t *__restrict__ lv, int64_t bL,
                                                int64_t nb, const K *__restrict__ rk,
                                                const int64_t *__restrict__ rv, int64_t bR,
                                                int64_t eR, const Place &pl, int64_t s, int &cp,
                                                int64_t &cb, const ProbeOut &o,
                                                int32_t *status, const JoinLds &L)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    K *out_key = (K *)o.key;
    const int64_t nbatch = (eR - bR + kJoinBatch - 1) / kJoinBatch;
    K kk[kJoinRows];
    int64_t vv[kJoinRows];
    uint32_t mf[kJoinRows];

    constexpr int64_t kCap = G::cap;
    if (CHUNKED && nb > kCap && nbatch > 0) {
        const int64_t nch = (nb + kCap - 1) / kCap;
        int64_t total = 0;
        for (int64_t c = 0; c < nch; ++c) {
            const int64_t c0 = c * kCap;
            build_table<G>(lk, lv, bL + c0, nb - c0 < kCap ? nb - c0 : kCap, L.tkey, L.tp, L.tn,
                           L.head);
            for (int64_t b = 0; b < nbatch; ++b) {
                load_batch(rk, rv, bR + b * kJoinBatch, eR, kk, vv);
                match_batch<G>(bR + b * kJoinBatch, eR, true, L.tkey, L.tn, L.head, kk, mf);
                cell_sums(mf, L.cw, lane, wv);
                __syncthreads();
                if (wv == 0) {
                    const int64_t all = cell_total(L.cw, lane);
                    if (lane == 0)
                        *L.s_total = all;
                }
                __syncthreads();
                total += *L.s_total;
            }
        }
        if (wv == 0) {
            const int64_t ex = place_rows(pl, s, total, cp, cb, lane, status);
            if (lane == 0)
                *L.s_excl = ex;
        }
        __syncthreads();
        const int64_t E = *L.s_excl;
        if (E + total > o.cap) {
            if (tid == 0 && total > 0)
                or_status(status, MDX_DEV_OUTPUT_OVERFLOW);
            return;
        }
        int64_t run = E;
        for (int64_t c = 0; c < nch && total > 0; ++c) {
            const int64_t c0 = c * kCap;
            build_table<G>(lk, lv, bL + c0, nb - c0 < kCap ? nb - c0 : kCap, L.tkey, L.tp, L.tn,
                           L.head);
            for (int64_t b = 0; b < nbatch; ++b) {
                load_batch(rk, rv, bR + b * kJoinBatch, eR, kk, vv);
                match_batch<G>(bR + b * kJoinBatch, eR, true, L.tkey, L.tn, L.head, kk, mf);
                cell_sums(mf, L.cw, lane, wv);
                __syncthreads();
                if (wv == 0) {
                    const int64_t all = cell_scan(L.cw, lane);
                    if (lane == 0)
                        *L.s_total = all;
                }
                __syncthreads();
                emit_batch<G>(kk, vv, mf, L.cw, run, L.tkey, L.tp, L.tn, out_key, o.lpay, o.rpay,
                              lane, wv);
                run += *L.s_total;
                __syncthreads();  // cw, s_total and the table are reused
            }
        }
        return;
    }

    if (nb > 0 && nb <= kCap && nbatch == 1) {
        join_one_batch<G, K>(lk, lv, bL, nb, rk, rv, bR, eR, pl, s, cp, cb, o, status, L);
        return;
    }

    // Any other sub-bucket (no build rows, no probe rows, or probe rows
    // beyond one batch).
    const bool any = nb > 0 && nbatch > 0;
    if (any)
        build_table<G>(lk, lv, bL, nb, L.tkey, L.tp, L.tn, L.head);

    // Count every probe row's matches.
    int64_t total = 0;
    for (int64_t b = 0; b < nbatch; ++b) {
        load_batch(rk, rv, bR + b * kJoinBatch, eR, kk, vv);
        match_batch<G>(bR + b * kJoinBatch, eR, any, L.tkey, L.tn, L.head, kk, mf);
        cell_sums(mf, L.cw, lane, wv);
        __syncthreads();
        if (wv == 0) {
            const int64_t all = cell_total(L.cw, lane);
            if (lane == 0)
                *L.s_total = all;
        }
        __syncthreads();
        total += *L.s_total;
    }

    // Output rows from the partition's cursor.
    if (wv == 0) {
        const int64_t ex = place_rows(pl, s, total, cp, cb, lane, status);
        if (lane == 0)
            *L.s_excl = ex;
    }
    __syncthreads();
    const int64_t E = *L.s_excl;

    // Write the output rows.
    if (E + total > o.cap) {
        if (tid == 0 && total > 0)
            or_status(status, MDX_DEV_OUTPUT_OVERFLOW);
    } else if (total > 0) {
        if (nbatch == 1) {
            if (wv == 0)
                cell_scan(L.cw, lane);
            __syncthreads();
            emit_batch<G>(kk, vv, mf, L.cw, E, L.tkey, L.tp, L.tn, out_key, o.lpay, o.rpay, lane,
                          wv);
        } else {
            int64_t run = E;
            for (int64_t b = 0; b < nbatch; ++b) {
                load_batch(rk, rv, bR + b * kJoinBatch, eR, kk, vv);
                match_batch<G>(bR + b * kJoinBatch, eR, any, L.tkey, L.tn, L.head, kk, mf);
                cell_sums(mf, L.cw, lane, wv);
                __syncthreads();
                if (wv == 0) {
                    const int64_t all = cell_scan(L.cw, lane);
                    if (lane == 0)
                        *L.s_total = all;
                }
                __syncthreads();
                emit_batch<G>(kk, vv, mf, L.cw, run, L.tkey, L.tp, L.tn, out_key, o.lpay, o.rpay,
                              lane, wv);
                run += *L.s_total;
                __syncthreads();  // cw and s_total are reused by the next batch
            }
        }
    }
}

// The kernel's kJoinPerCu workgroups of kJoinThreads fill a CU's 4 SIMDs
// with kJoinSimdWaves waves each.
constexpr int kJoinSimdWaves = kJoinPerCu * kJoinThreads / (4 * kWave);

// Sub-buckets are taken strictly in ticket order, just before each is
// started: a ticket taken ahead of time would make later sub-buckets wait
// for it in the chained scan.
#define MDX_JOIN_LDS(G)                                                                    \
    __shared__ int64_t tkey[G::cap + 1];                                                   \
    __shared__ int64_t tp[G::cap];                                                         \
    __shared__ uint16_t tn[G::cap + 1];                                                    \
    __shared__ uint32_t head[G::heads];                                                    \
    __shared__ int64_t cw[kCells];                                                         \
    __shared__ int64_t s_next, s_excl, s_total;                                            \
    const JoinLds L = {tkey, tp, tn, head, cw, &s_excl, &s_total};                         \
    if (threadIdx.x == 0) {                                                                \
        tkey[G::cap] = 0;                                                                  \
        tn[G::cap] = (uint16_t)G::cap;                                                     \
    }

// Next ticket, the same on every lane.
__device__ __forceinline__ int64_t take_ticket(uint32_t *ticket, int64_t *s_next)
{
    if (threadIdx.x == 0)
        *s_next = (int64_t)atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t t = uniform(*s_next);
    __syncthreads();  // everyone has read s_next before it is replaced
    return t;
}

// CHUNKED: oversized build sub-buckets are joined in chunks; otherwise the
// kernel does nothing unless the plan found that every one fits a table.
template <typename K, bool CHUNKED>
__global__ __launch_bounds__(kJoinThreads)
__attribute__((amdgpu_waves_per_eu(kJoinSimdWaves, kJoinSimdWaves))) void rj_join(
    const K *__restrict__ lk, const int64_t *__restrict__ lv, const int64_t *__restrict__ subL,
    const K *__restrict__ rk, const int64_t *__restrict__ rv, const int64_t *__restrict__ subR,
    RJoinWs w, int qbits, int by_part, ProbeOut o, int32_t *status)
{
    if (!CHUNKED && *w.use == 0)
        return;
    MDX_JOIN_LDS(MergeJoin)
    const int64_t S = w.S;
    const Place pl = {(uint64_t *)w.tile_base, w.status, qbits, by_part};
    int cp = -1;
    int64_t cb = 0;
    for (;;) {
        const int64_t s = take_ticket(w.ticket, &s_next);
        if (s >= S)
            break;
        const int64_t bL = subL[s], nb = subL[s + 1] - bL;
        join_sub_bucket<MergeJoin, K, CHUNKED>(lk, lv, bL, nb, rk, rv, subR[s], subR[s + 1], pl,
                                               s, cp, cb, o, status, L);
        __syncthreads();  // the table is reused by the next sub-bucket
    }
}

// Every merge of a batch: tickets run over all merges' sub-buckets (merge m
// owns tickets [Spre[m], Spre[m+1])), so the workgroups stay busy across
// merges; each merge has its own partition cursors and chained scan.
template <typename K>
__global__ __launch_bounds__(kJoinThreads)
__attribute__((amdgpu_waves_per_eu(kJoinSimdWaves, kJoinSimdWaves))) void rj_join_batch(
    const JoinRec *__restrict__ B, const uint32_t *__restrict__ Spre, int M, uint32_t *ticket)
{
    MDX_JOIN_LDS(BatchJoin)
    const int64_t total = Spre[M];
    int64_t c0 = 0, c1 = 0;  // tickets of the merge whose record is loaded
    JoinRec r = {};
    int cp = -1;  // place_rows' cache, per merge
    int64_t cb = 0;
    for (;;) {
        const int64_t t = take_ticket(ticket, &s_next);
        if (t >= total)
            break;
        if (t < c0 || t >= c1) {
            const int m = find_range(Spre, M, (uint32_t)t);
            c0 = Spre[m];
            c1 = Spre[m + 1];
            r = B[m];
            cp = -1;
        }
        const int64_t s = t - c0;
        const int64_t *subL = r.subL, *subR = r.subR;
        const int64_t bL = subL[s];
        const Place pl = {(uint64_t *)r.jbase, r.jstatus, r.qbits, r.by_part};
        join_sub_bucket<BatchJoin, K, true>((const K *)r.lk, r.lv, bL, subL[s + 1] - bL, (const K *)r.rk,
                                 r.rv, subR[s], subR[s + 1], pl, s, cp, cb, r.o, r.status, L);
        __syncthreads();  // the table is reused by the next sub-bucket
    }
}

// Block m: clear merge m's partition cursors and chained scan.  Block 0
// also resets the ticket.
__global__ __launch_bounds__(kBlock) void rj_clear_batch(const JoinRec *__restrict__ B,
                                                         uint32_t *ticket)
{
    const JoinRec &r = B[blockIdx.x];
    for (int64_t s = threadIdx.x; s < r.S; s += kBlock) {
        r.jstatus[s] = 0;
        r.jbase[s] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *ticket = 0;
}

// offsets[0..P] from the placement, one block: by sub-bucket, the first
// output row of each partition's first sub-bucket and the scan's total; by
// partition, the exclusive prefix of the partition totals (the rows each
// partition's cursor took).
__device__ inline void offsets_from_place(const uint64_t *part, const uint64_t *pst, int P,
                                          int qbits, int64_t S, bool by_part, int64_t *offsets)
{
    if (!by_part) {
        const int64_t total = (int64_t)(ld_agent(pst + S - 1) & kValMask);
        for (int p = threadIdx.x; p <= P; p += kBlock)
            offsets[p] = p < P ? (int64_t)part[(int64_t)p << qbits] : total;
        return;
    }
    __shared__ int64_t scratch[kWavesPerBlock];
    int64_t carry = 0;
    for (int b = 0; b < P; b += kBlock) {
        const int p = b + threadIdx.x;
        const int64_t v = p < P ? (int64_t)(ld_agent(part + p) >> kDoneBits) : 0;
        int64_t all;
        const int64_t ex = block_excl_scan(v, scratch, &all);
        if (p < P)
            offsets[p] = carry + ex;
        carry += all;
    }
    if (threadIdx.x == 0)
        offsets[P] = carry;
}

// Block m: merge m's output offsets.
__global__ __launch_bounds__(kBlock) void rj_finalize_batch(const JoinRec *__restrict__ B)
{
    const JoinRec &r = B[blockIdx.x];
    offsets_from_place((const uint64_t *)r.jbase, r.jstatus, r.P, r.qbits, r.S, r.by_part != 0,
                       r.o.offsets);
}

// Output offsets of a merge: from the radix join's partition cursors when it
// ran (*w.use), else from the global-table probe's chained scan (probe tiles,
// partition-major).
__global__ __launch_bounds__(kBlock) void merge_finalize(int P, int qbits, int by_part, RJoinWs w,
                                                         ProbeWs pw, bool fallback, ProbeOut o)
{
    if (*w.use != 0) {
        offsets_from_place((const uint64_t *)w.tile_base, w.status, P, qbits, w.S, by_part != 0,
                           o.offsets);
    } else if (fallback) {
        const int64_t TT = pw.tile_start[P];
        const int64_t total = TT > 0 ? (int64_t)(ld_agent(pw.status + TT - 1) & kValMask) : 0;
        for (int p = threadIdx.x; p <= P; p += kBlock) {
            const int64_t t = pw.tile_start[p];
            o.offsets[p] = t < TT ? pw.tile_base[t] : total;
        }
    }
}

}  // namespace

int rjoin_grid(int64_t S)
{
    // kJoinPerCu workgroups per CU (all resident at once), or one per
    // sub-bucket when there are fewer: a workgroup holds half a CU's LDS,
    // which other merges' kernels may need meanwhile.
    const int64_t cus = device_fill_blocks() / 8 > 0 ? device_fill_blocks() / 8 : 1;
    return (int)std::max<int64_t>(1, std::min<int64_t>(cus * kJoinPerCu, S));
}

bool rjoin_by_partition(int qbits, int64_t G)
{
    return ((int64_t)1 << qbits) >= 8 * G;
}

hipError_t launch_rjoin_plan(const int64_t *subL, const int64_t *subR, int64_t S,
                             const RJoinWs &w, bool chunked, hipStream_t s)
{
    (void)subR;
    if (S <= kPlanOneMax) {
        hipLaunchKernelGGL(rj_plan_one, dim3(1), dim3(kBlock), 0, s, subL, S, w, (int)chunked);
        return hipGetLastError();
    }
    const int64_t cus = device_fill_blocks() / 8 > 0 ? device_fill_blocks() / 8 : 1;
    const int G = (int)std::min<int64_t>(cus, (S + kBlock - 1) / kBlock + 1);
    hipLaunchKernelGGL(rj_plan_init, dim3(1), dim3(1), 0, s, w);
    hipLaunchKernelGGL(rj_plan, dim3(G), dim3(kBlock), 0, s, subL, S, w, (int)chunked);
    return hipGetLastError();
}

template <bool CHUNKED>
void launch_rjoin_kernel(int G, const void *lk, const int64_t *lv, const int64_t *subL,
                         const void *rk, const int64_t *rv, const int64_t *subR, int key_bytes,
                         const RJoinWs &w, int qbits, const ProbeOut &o, int32_t *status,
                         hipStream_t s)
{
    const int by_part = rjoin_by_partition(qbits, G) ? 1 : 0;
    if (key_bytes == 8)
        hipLaunchKernelGGL((rj_join<int64_t, CHUNKED>), dim3(G), dim3(kJoinThreads), 0, s,
                           (const int64_t *)lk, lv, subL, (const int64_t *)rk, rv, subR, w, qbits,
                           by_part, o, status);
    else
        hipLaunchKernelGGL((rj_join<int32_t, CHUNKED>), dim3(G), dim3(kJoinThreads), 0, s,
                           (const int32_t *)lk, lv, subL, (const int32_t *)rk, rv, subR, w, qbits,
                           by_part, o, status);
}

hipError_t launch_rjoin(const void *lk, const int64_t *lv, const int64_t *subL, const void *rk,
                        const int64_t *rv, const int64_t *subR, int key_bytes, int32_t P,
                        int qbits, const RJoinWs &w, const ProbeOut &o, int32_t *status,
                        bool chunked, hipStream_t s)
{
    (void)P;
    const int G = rjoin_grid(w.S);
    trace_begin("rj_join", s);
    if (chunked)
        launch_rjoin_kernel<true>(G, lk, lv, subL, rk, rv, subR, key_bytes, w, qbits, o, status,
                                  s);
    else
        launch_rjoin_kernel<false>(G, lk, lv, subL, rk, rv, subR, key_bytes, w, qbits, o, status,
                                   s);
    trace_end("rj_join", s);
    return hipGetLastError();
}

hipError_t launch_rjoin_batch(const JoinRec *recs, int M, const uint32_t *Spre, uint32_t S,
                              uint32_t *ticket, int key_bytes, hipStream_t s)
{
    if (M <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(rj_clear_batch, dim3((unsigned)M), dim3(kBlock), 0, s, recs, ticket);
    const int G = rjoin_grid(S);
    trace_begin("rj_join", s);
    if (key_bytes == 8)
        hipLaunchKernelGGL(rj_join_batch<int64_t>, dim3(G), dim3(kJoinThreads), 0, s, recs, Spre,
                           M, ticket);
    else
        hipLaunchKernelGGL(rj_join_batch<int32_t>, dim3(G), dim3(kJoinThreads), 0, s, recs, Spre,
                           M, ticket);
    trace_end("rj_join", s);
    hipLaunchKernelGGL(rj_finalize_batch, dim3((unsigned)M), dim3(kBlock), 0, s, recs);
    return hipGetLastError();
}

hipError_t launch_merge_finalize(int32_t P, int qbits, const RJoinWs &w, const ProbeWs *pw,
                                 const ProbeOut &o, hipStream_t s)
{
    const ProbeWs none = {};
    const int by_part = rjoin_by_partition(qbits, rjoin_grid(w.S)) ? 1 : 0;
    hipLaunchKernelGGL(merge_finalize, dim3(1), dim3(kBlock), 0, s, P, qbits, by_part, w,
                       pw ? *pw : none, pw != nullptr, o);
    return hipGetLastError();
}

}  // namespace mdx
