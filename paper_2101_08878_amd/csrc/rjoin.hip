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
//   2. streams the probe rows in chunks of 4096, counts each row's matches by
//      walking its chain, obtains the output rows of every earlier chunk from
//      a chained scan (decoupled look-back over chunks in sub-bucket order),
//      and writes (key, left payload, right payload) rows.
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
constexpr int kBuildBatch = 4;

// Chain bucket: hash bits 20..31, away from the partition's low bits and the
// sub-bucket's top bits.
__device__ __forceinline__ uint32_t bucket_of(uint64_t h)
{
    return (uint32_t)(h >> 20) & (kJoinHeads - 1);
}

__global__ __launch_bounds__(kBlock) void rj_plan(const int64_t *__restrict__ subL,
                                                  const int64_t *__restrict__ subR, int64_t S,
                                                  RJoinWs w)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    if (blockIdx.x == 0) {
        int64_t carry = 0;
        int over = 0;
        for (int64_t base = 0; base < S; base += kBlock) {
            const int64_t s = base + threadIdx.x;
            int64_t nc = 0;
            if (s < S) {
                nc = (subR[s + 1] - subR[s] + kJoinChunk - 1) / kJoinChunk;
                over |= (subL[s + 1] - subL[s]) > kJoinCap;
            }
            int64_t tot;
            const int64_t ex = block_excl_scan(nc, scratch, &tot);
            if (s < S)
                w.chunk_start[s] = carry + ex;
            carry += tot;
        }
        over = __syncthreads_or(over);
        if (threadIdx.x == 0) {
            w.chunk_start[S] = carry;
            *w.use = over ? 0 : 1;
            *w.ticket = 0;
        }
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < w.max_chunks; i += stride)
        w.status[i] = 0;
}

template <typename K>
__global__ __launch_bounds__(kJoinThreads) void rj_join(
    const K *__restrict__ lk, const int64_t *__restrict__ lv, const int64_t *__restrict__ subL,
    const K *__restrict__ rk, const int64_t *__restrict__ rv, const int64_t *__restrict__ subR,
    int64_t S, RJoinWs w, ProbeOut o, int32_t *status)
{
    __shared__ uint64_t th[kJoinCap];     // hash of build row i
    __shared__ int64_t tp[kJoinCap];      // payload of build row i
    __shared__ uint16_t tn[kJoinCap];     // next row in i's chain
    __shared__ uint32_t head[kJoinHeads]; // last row inserted per bucket
    __shared__ int64_t cw[kJoinRows][kJoinWaves];
    __shared__ int64_t s_sb, s_excl, s_total;
    static_assert(kJoinRows * kJoinWaves == kWave, "one wave scans the chunk's partial sums");

    if (*w.use == 0)
        return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    K *out_key = (K *)o.key;

    for (;;) {
        if (tid == 0)
            s_sb = (int64_t)atomicAdd(w.ticket, 1u);
        __syncthreads();
        const int64_t s = s_sb;
        if (s >= S)
            break;
        const int64_t c0 = w.chunk_start[s], nch = w.chunk_start[s + 1] - c0;
        if (nch > 0) {
            const int64_t bL = subL[s], nb = subL[s + 1] - bL;  // nb <= kJoinCap (plan flag)
            const int64_t bR = subR[s], eR = subR[s + 1];

            // 1. build, kBuildBatch rows per thread at a time
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

            // 2. probe, chunk by chunk
            for (int64_t c = 0; c < nch; ++c) {
                const int64_t tile = c0 + c;
                const int64_t rbase = bR + c * kJoinChunk;
                K kk[kJoinRows];
                int64_t vv[kJoinRows];
                uint64_t hh[kJoinRows];
                uint32_t first[kJoinRows], m[kJoinRows];
#pragma unroll
                for (int j = 0; j < kJoinRows; ++j) {
                    const int64_t r = rbase + (int64_t)j * kJoinThreads + tid;
                    kk[j] = r < eR ? __builtin_nontemporal_load(rk + r) : K(0);
                    vv[j] = r < eR ? __builtin_nontemporal_load(rv + r) : 0;
                }
#pragma unroll
                for (int j = 0; j < kJoinRows; ++j) {
                    const int64_t r = rbase + (int64_t)j * kJoinThreads + tid;
                    m[j] = 0;
                    first[j] = kNil;
                    hh[j] = fmix64(key_bits(kk[j]));
                    if (r < eR) {
                        uint32_t e = head[bucket_of(hh[j])];
                        while (e != kNil) {
                            if (th[e] == hh[j]) {
                                if (m[j] == 0)
                                    first[j] = e;
                                ++m[j];
                            }
                            const uint16_t nx = tn[e];
                            e = nx == kNil16 ? kNil : (uint32_t)nx;
                        }
                    }
                }
                // output rank of every row: order (j, thread) = row order
                int64_t mex[kJoinRows];
#pragma unroll
                for (int j = 0; j < kJoinRows; ++j) {
                    const int64_t inc = wave_incl_scan((int64_t)m[j], lane);
                    mex[j] = inc - (int64_t)m[j];
                    if (lane == kWave - 1)
                        cw[j][wv] = inc;
                }
                __syncthreads();
                // Wave 0: exclusive scan of the 64 (row step, wave) sums in
                // place, then the chained scan for the chunk's total.
                if (wv == 0) {
                    int64_t *flat = &cw[0][0];
                    const int64_t x = flat[lane];
                    const int64_t inc = wave_incl_scan(x, lane);
                    flat[lane] = inc - x;
                    const int64_t M = __shfl(inc, kWave - 1, kWave);
                    const int64_t ex = lookback(w.status, tile, M, lane, status);
                    if (lane == 0) {
                        s_excl = ex;
                        s_total = M;
                        w.tile_base[tile] = ex;
                    }
                }
                __syncthreads();
                const int64_t E = s_excl, M = s_total;
                int64_t cbase[kJoinRows];
#pragma unroll
                for (int j = 0; j < kJoinRows; ++j)
                    cbase[j] = cw[j][wv];
                if (E + M > o.cap) {
                    if (tid == 0 && M > 0)
                        or_status(status, MDX_DEV_OUTPUT_OVERFLOW);
                } else {
#pragma unroll
                    for (int j = 0; j < kJoinRows; ++j) {
                        if (m[j] == 0)
                            continue;
                        int64_t at = E + cbase[j] + mex[j];
                        if (m[j] == 1) {
                            out_key[at] = kk[j];
                            o.lpay[at] = tp[first[j]];
                            o.rpay[at] = vv[j];
                        } else {
                            uint32_t e = first[j];
                            while (e != kNil) {
                                if (th[e] == hh[j]) {
                                    out_key[at] = kk[j];
                                    o.lpay[at] = tp[e];
                                    o.rpay[at] = vv[j];
                                    ++at;
                                }
                                const uint16_t nx = tn[e];
                                e = nx == kNil16 ? kNil : (uint32_t)nx;
                            }
                        }
                    }
                }
                __syncthreads();  // cw and s_excl are reused by the next chunk
            }
        }
        __syncthreads();  // the table is reused by the next sub-bucket
    }
}

__global__ __launch_bounds__(kBlock) void rj_finalize(int P, int qbits, RJoinWs w, ProbeOut o)
{
    if (*w.use == 0)
        return;
    const int64_t S = (int64_t)P << qbits;
    const int64_t TT = w.chunk_start[S];
    const int64_t total = TT > 0 ? (int64_t)(ld_agent(w.status + TT - 1) & kValMask) : 0;
    for (int p = threadIdx.x; p <= P; p += kBlock) {
        const int64_t t = w.chunk_start[(int64_t)p << qbits];
        o.offsets[p] = t < TT ? w.tile_base[t] : total;
    }
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
    const int G = device_fill_blocks() / 8 > 0 ? device_fill_blocks() / 8 : 1;
    hipLaunchKernelGGL(rj_plan, dim3(G), dim3(kBlock), 0, s, subL, subR, S, w);
    return hipGetLastError();
}

hipError_t launch_rjoin(const void *lk, const int64_t *lv, const int64_t *subL, const void *rk,
                        const int64_t *rv, const int64_t *subR, int key_bytes, int32_t P,
                        int qbits, const RJoinWs &w, const ProbeOut &o, int32_t *status,
                        hipStream_t s)
{
    const int64_t S = (int64_t)P << qbits;
    const int G = device_fill_blocks() / 8 > 0 ? device_fill_blocks() / 8 : 1;  // one per CU
    trace_begin("rj_join", s);
    if (key_bytes == 8)
        hipLaunchKernelGGL(rj_join<int64_t>, dim3(G), dim3(kJoinThreads), 0, s,
                           (const int64_t *)lk, lv, subL, (const int64_t *)rk, rv, subR, S, w, o,
                           status);
    else
        hipLaunchKernelGGL(rj_join<int32_t>, dim3(G), dim3(kJoinThreads), 0, s,
                           (const int32_t *)lk, lv, subL, (const int32_t *)rk, rv, subR, S, w, o,
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
