// Radix join: the per-partition inner join (arXiv 2101.08878, Section V-B
// "cuDF Merge": every worker merges the frames it received) with every table
// held in LDS.
//
// Both sides arrive split into sub-buckets (partition p, top hash bits q), so
// that a sub-bucket's build rows fit one workgroup's LDS.  A workgroup takes
// sub-buckets in order from a ticket counter; for each it
//   1. loads the build rows into LDS: full 64-bit hash, payload, and a chain
//      link; bucket heads hold the last row inserted per bucket (LDS atomic
//      exchange), so equal keys share a chain and repeated keys need nothing
//      special (fmix64 is a bijection: equal hashes are equal keys);
//   2. counts the output rows of all its probe rows (walking each row's
//      chain), publishes that count to a chained scan over sub-buckets
//      (decoupled look-back), and receives the output rows of all earlier
//      sub-buckets;
//   3. writes (key, left payload, right payload) rows.  When the probe rows
//      fit one batch (8192 rows) they stay in registers between 2 and 3;
//      otherwise they are read and looked up again.
// Sub-buckets are numbered partition-major, so partition p's output is the
// contiguous range [out_off[p], out_off[p+1]).  Global memory is only
// streamed: the random accesses of the join all hit LDS.
#include "mdx.h"
#include "mdx_internal.hpp"

namespace mdx {
namespace {

constexpr uint32_t kNil = 0xffffffffu;
constexpr uint16_t kNil16 = 0xffffu;
constexpr int kJoinWaves = kJoinThreads / kWave;
constexpr int kBuildBatch = 8;
constexpr int kCells = kJoinRows * kJoinWaves;  // (row step, wave) partial sums
constexpr int kCellsPerLane = kCells / kWave;
static_assert(kCells % kWave == 0, "one wave scans the partial sums");

// Chain bucket: hash bits 20..31, away from the partition's low bits and the
// sub-bucket's top bits.
__device__ __forceinline__ uint32_t bucket_of(uint64_t h)
{
    return (uint32_t)(h >> 20) & (kJoinHeads - 1);
}

__global__ __launch_bounds__(kBlock) void rj_plan(const int64_t *__restrict__ subL, int64_t S,
                                                  RJoinWs w)
{
    int over = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < S; s += stride) {
        w.status[s] = 0;
        over |= (subL[s + 1] - subL[s]) > kJoinCap;
    }
    if (over)
        *w.use = 0;  // any block may clear it; block 0 set it below first
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *w.ticket = 0;
}

__global__ void rj_plan_init(RJoinWs w)
{
    *w.use = 1;
}

// Look up rows [rb, re) of the probe side (this thread's rows: rb + j * 1024
// + tid): per row the number of matches (high 16 bits; at most kJoinCap) and
// the first matching build row (low 16 bits).
template <typename K>
__device__ __forceinline__ void lookup_batch(const K *__restrict__ rk, const int64_t *__restrict__ rv,
                                             int64_t rb, int64_t re, bool any, const uint64_t *th,
                                             const uint16_t *tn, const uint32_t *head, K *kk,
                                             int64_t *vv, uint32_t *mf)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kJoinRows; ++j) {
        const int64_t r = rb + (int64_t)j * kJoinThreads + tid;
        kk[j] = r < re ? __builtin_nontemporal_load(rk + r) : K(0);
        vv[j] = r < re ? __builtin_nontemporal_load(rv + r) : 0;
    }
#pragma unroll
    for (int j = 0; j < kJoinRows; ++j) {
        const int64_t r = rb + (int64_t)j * kJoinThreads + tid;
        uint32_t cnt = 0, fst = kNil16;
        if (any && r < re) {
            const uint64_t h = fmix64(key_bits(kk[j]));
            uint32_t e = head[bucket_of(h)];
            while (e != kNil) {
                if (th[e] == h) {
                    if (cnt == 0)
                        fst = e;
                    ++cnt;
                }
                const uint16_t nx = tn[e];
                e = nx == kNil16 ? kNil : (uint32_t)nx;
            }
        }
        mf[j] = (cnt << 16) | fst;
    }
}

// Per-(row step, wave) sums of m into cw (row order = step-major).
__device__ __forceinline__ void cell_sums(const uint32_t *mf, int64_t *cw, int lane, int wv)
{
#pragma unroll
    for (int j = 0; j < kJoinRows; ++j) {
        const int64_t s = wave_sum((int64_t)(mf[j] >> 16));
        if (lane == 0)
            cw[j * kJoinWaves + wv] = s;
    }
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
template <typename K>
__device__ __forceinline__ void emit_batch(const K *kk, const int64_t *vv, const uint32_t *mf,
                                           const int64_t *cw, int64_t base,
                                           const uint64_t *th, const int64_t *tp,
                                           const uint16_t *tn, K *out_key, int64_t *out_l,
                                           int64_t *out_r, int lane, int wv)
{
#pragma unroll
    for (int j = 0; j < kJoinRows; ++j) {
        const uint32_t cnt = mf[j] >> 16, fst = mf[j] & 0xffffu;
        const int64_t inc = wave_incl_scan((int64_t)cnt, lane);
        if (cnt == 0)
            continue;
        int64_t at = base + cw[j * kJoinWaves + wv] + inc - (int64_t)cnt;
        if (cnt == 1) {
            out_key[at] = kk[j];
            out_l[at] = tp[fst];
            out_r[at] = vv[j];
        } else {
            const uint64_t h = fmix64(key_bits(kk[j]));
            uint32_t e = fst;
            while (e != kNil) {
                if (th[e] == h) {
                    out_key[at] = kk[j];
                    out_l[at] = tp[e];
                    out_r[at] = vv[j];
                    ++at;
                }
                const uint16_t nx = tn[e];
                e = nx == kNil16 ? kNil : (uint32_t)nx;
            }
        }
    }
}

template <typename K>
__global__ __launch_bounds__(kJoinThreads) void rj_join(
    const K *__restrict__ lk, const int64_t *__restrict__ lv, const int64_t *__restrict__ subL,
    const K *__restrict__ rk, const int64_t *__restrict__ rv, const int64_t *__restrict__ subR,
    RJoinWs w, ProbeOut o, int32_t *status)
{
    __shared__ uint64_t th[kJoinCap];     // hash of build row i
    __shared__ int64_t tp[kJoinCap];      // payload of build row i
    __shared__ uint16_t tn[kJoinCap];     // next row in i's chain
    __shared__ uint32_t head[kJoinHeads]; // last row inserted per bucket
    __shared__ int64_t cw[kCells];
    __shared__ int64_t s_sb, s_excl, s_total;

    if (*w.use == 0)
        return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    K *out_key = (K *)o.key;
    const int64_t S = w.S;

    for (;;) {
        if (tid == 0)
            s_sb = (int64_t)atomicAdd(w.ticket, 1u);
        __syncthreads();
        const int64_t s = s_sb;
        if (s >= S)
            break;
        const int64_t bL = subL[s], nb = subL[s + 1] - bL;  // nb <= kJoinCap (plan flag)
        const int64_t bR = subR[s], eR = subR[s + 1];
        const int64_t nbatch = (eR - bR + kJoinBatch - 1) / kJoinBatch;
        const bool any = nb > 0 && nbatch > 0;

        // 1. build, kBuildBatch rows per thread at a time
        if (any) {
            for (int i = tid; i < kJoinHeads; i += kJoinThreads)
                head[i] = kNil;
            __syncthreads();
            for (int base = 0; base < (int)nb; base += kBuildBatch * kJoinThreads) {
                K bk[kBuildBatch];
                int64_t bv[kBuildBatch];
#pragma unroll
                for (int j = 0; j < kBuildBatch; ++j) {
                    const int i = base + j * kJoinThreads + tid;
                    bk[j] = i < nb ? __builtin_nontemporal_load(lk + bL + i) : K(0);
                    bv[j] = i < nb ? __builtin_nontemporal_load(lv + bL + i) : 0;
                }
#pragma unroll
                for (int j = 0; j < kBuildBatch; ++j) {
                    const int i = base + j * kJoinThreads + tid;
                    if (i < nb) {
                        const uint64_t h = fmix64(key_bits(bk[j]));
                        th[i] = h;
                        tp[i] = bv[j];
                        tn[i] = (uint16_t)atomicExch(&head[bucket_of(h)], (uint32_t)i);
                    }
                }
            }
            __syncthreads();
        }

        // 2. count every probe row's matches
        K kk[kJoinRows];
        int64_t vv[kJoinRows];
        uint32_t mf[kJoinRows];
        int64_t total = 0;
        for (int64_t b = 0; b < nbatch; ++b) {
            lookup_batch(rk, rv, bR + b * kJoinBatch, eR, any, th, tn, head, kk, vv, mf);
            cell_sums(mf, cw, lane, wv);
            __syncthreads();
            if (wv == 0) {
                int64_t loc = 0;
#pragma unroll
                for (int i = 0; i < kCellsPerLane; ++i)
                    loc += cw[lane * kCellsPerLane + i];
                const int64_t all = wave_sum(loc);
                if (lane == 0)
                    s_total = all;
            }
            __syncthreads();
            total += s_total;
        }

        // chained scan over sub-buckets
        if (wv == 0) {
            const int64_t ex = lookback(w.status, s, total, lane, status);
            if (lane == 0) {
                s_excl = ex;
                w.tile_base[s] = ex;
            }
        }
        __syncthreads();
        const int64_t E = s_excl;

        // 3. write the output rows
        if (E + total > o.cap) {
            if (tid == 0 && total > 0)
                or_status(status, MDX_DEV_OUTPUT_OVERFLOW);
        } else if (total > 0) {
            if (nbatch == 1) {
                if (wv == 0)
                    cell_scan(cw, lane);
                __syncthreads();
                emit_batch(kk, vv, mf, cw, E, th, tp, tn, out_key, o.lpay, o.rpay, lane, wv);
            } else {
                int64_t run = E;
                for (int64_t b = 0; b < nbatch; ++b) {
                    lookup_batch(rk, rv, bR + b * kJoinBatch, eR, any, th, tn, head, kk, vv, mf);
                    cell_sums(mf, cw, lane, wv);
                    __syncthreads();
                    if (wv == 0) {
                        const int64_t all = cell_scan(cw, lane);
                        if (lane == 0)
                            s_total = all;
                    }
                    __syncthreads();
                    emit_batch(kk, vv, mf, cw, run, th, tp, tn, out_key, o.lpay, o.rpay, lane, wv);
                    run += s_total;
                    __syncthreads();  // cw and s_total are reused by the next batch
                }
            }
        }
        __syncthreads();  // the table is reused by the next sub-bucket
    }
}

__global__ __launch_bounds__(kBlock) void rj_finalize(int P, int qbits, RJoinWs w, ProbeOut o)
{
    if (*w.use == 0)
        return;
    const int64_t S = w.S;
    const int64_t total = (int64_t)(ld_agent(w.status + S - 1) & kValMask);
    for (int p = threadIdx.x; p <= P; p += kBlock)
        o.offsets[p] = p < P ? w.tile_base[(int64_t)p << qbits] : total;
}

__global__ __launch_bounds__(kBlock) void gather_offsets(const int64_t *__restrict__ a, int P,
                                                         int stride, int64_t *__restrict__ out)
{
    for (int p = threadIdx.x; p <= P; p += kBlock)
        out[p] = a[(int64_t)p * stride];
}

}  // namespace

hipError_t launch_rjoin_plan(const int64_t *subL, const int64_t *subR, int64_t S,
                             const RJoinWs &w, hipStream_t s)
{
    (void)subR;
    const int G = device_fill_blocks() / 8 > 0 ? device_fill_blocks() / 8 : 1;
    hipLaunchKernelGGL(rj_plan_init, dim3(1), dim3(1), 0, s, w);
    hipLaunchKernelGGL(rj_plan, dim3(G), dim3(kBlock), 0, s, subL, S, w);
    return hipGetLastError();
}

hipError_t launch_rjoin(const void *lk, const int64_t *lv, const int64_t *subL, const void *rk,
                        const int64_t *rv, const int64_t *subR, int key_bytes, int32_t P,
                        int qbits, const RJoinWs &w, const ProbeOut &o, int32_t *status,
                        hipStream_t s)
{
    (void)P;
    (void)qbits;
    const int G = device_fill_blocks() / 8 > 0 ? device_fill_blocks() / 8 : 1;  // one per CU
    trace_begin("rj_join", s);
    if (key_bytes == 8)
        hipLaunchKernelGGL(rj_join<int64_t>, dim3(G), dim3(kJoinThreads), 0, s,
                           (const int64_t *)lk, lv, subL, (const int64_t *)rk, rv, subR, w, o,
                           status);
    else
        hipLaunchKernelGGL(rj_join<int32_t>, dim3(G), dim3(kJoinThreads), 0, s,
                           (const int32_t *)lk, lv, subL, (const int32_t *)rk, rv, subR, w, o,
                           status);
    trace_end("rj_join", s);
    return hipGetLastError();
}

hipError_t launch_rjoin_finalize(int32_t P, int qbits, const RJoinWs &w, const ProbeOut &o,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(rj_finalize, dim3(1), dim3(kBlock), 0, s, P, qbits, w, o);
    return hipGetLastError();
}

hipError_t launch_gather_offsets(const int64_t *a, int32_t P, int stride, int64_t *out,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(gather_offsets, dim3(1), dim3(kBlock), 0, s, a, P, stride, out);
    return hipGetLastError();
}

}  // namespace mdx
