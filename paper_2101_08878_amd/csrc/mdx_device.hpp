// Device helpers shared by the libmdx kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mdx.h"

namespace mdx {

constexpr int kWave = 64;
#ifndef MDX_BLOCK
#define MDX_BLOCK 512
#endif
constexpr int kBlock = MDX_BLOCK;      // threads per workgroup (8 waves)
constexpr int kWavesPerBlock = kBlock / kWave;

// ---- the hash -------------------------------------------------------------
// MurmurHash3's 64-bit finalizer: xor-shift 33, multiply, xor-shift 33,
// multiply, xor-shift 33 (all mod 2^64).  It is a bijection of uint64, so
// two keys are equal exactly when their hashes are; the tables store hashes.
__device__ __forceinline__ uint64_t fmix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

// Keys enter the hash as the bits of their int64 value (int32 sign-extends).
template <typename K>
__device__ __forceinline__ uint64_t key_bits(K k)
{
    return (uint64_t)(int64_t)k;
}

// Destination of a hash: the partition p = h mod P (unsigned; power-of-two P
// uses a mask), optionally refined by the top `sbits` bits of h into
// sub-bucket q: d = p * 2^sbits + q.  With sbits = 0 the destination is the
// partition itself.
struct Dest {
    uint64_t P;
    uint64_t mask;  // P - 1 when P is a power of two
    int32_t pow2;
    int32_t sbits;  // sub-bucket bits taken from the top of h
    int32_t ndest;  // P << sbits
    int32_t nbits;  // bits needed to write ndest - 1 (0 for ndest = 1)
};

__device__ __forceinline__ uint32_t part_of(uint64_t h, const Dest &d)
{
    return d.pow2 ? (uint32_t)(h & d.mask) : (uint32_t)(h % d.P);
}

__device__ __forceinline__ uint32_t dest_of(uint64_t h, const Dest &d)
{
    const uint32_t p = part_of(h, d);
    return d.sbits ? ((p << d.sbits) | (uint32_t)(h >> (64 - d.sbits))) : p;
}

// Bits [64 - shift - bits, 64 - shift) of h: the sub-bucket digit below the
// `shift` top bits already used.
__device__ __forceinline__ uint32_t digit_of(uint64_t h, int shift, int bits)
{
    return bits ? (uint32_t)((h << shift) >> (64 - bits)) : 0u;
}

// ---- wave primitives ------------------------------------------------------
__device__ __forceinline__ uint64_t ballot(bool p)
{
    return __builtin_amdgcn_ballot_w64(p);
}

// Number of set bits of m in lanes below the calling lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int lane_id()
{
    return (int)mbcnt(~0ull);
}

// Inclusive scan of a 64-bit value across the wave.
__device__ __forceinline__ int64_t wave_incl_scan(int64_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int64_t u = __shfl_up(v, (unsigned)d, kWave);
        if (lane >= d)
            v += u;
    }
    return v;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v)
{
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1)
        v += __shfl_xor(v, d, kWave);
    return v;
}

// Exclusive scan over a kBlock-thread block.  Returns the thread's exclusive
// prefix; *total receives the block sum.  Uses 4 int64 of LDS (scratch).
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *scratch, int64_t *total)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    int64_t inc = wave_incl_scan(v, lane);
    if (lane == kWave - 1)
        scratch[w] = inc;
    __syncthreads();
    int64_t before = 0, sum = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
        int64_t s = scratch[i];
        before += (i < w) ? s : 0;
        sum += s;
    }
    __syncthreads();
    *total = sum;
    return before + inc - v;
}

// Copy P+1 partition offsets, made safe to index with: out[p] =
// min(n, max(0, in[0..p])), a non-decreasing sequence inside [0, n].
// Offsets that were already valid are copied unchanged.  Whole block calls.
__device__ __forceinline__ void sanitize_offsets(const int64_t *in, int64_t *out, int P, int64_t n,
                                                 int64_t *scratch)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    int64_t carry = 0;
    for (int base = 0; base <= P; base += kBlock) {
        const int p = base + tid;
        int64_t v = p <= P ? in[p] : 0;
        v = v < 0 ? 0 : v;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int64_t u = __shfl_up(v, (unsigned)d, kWave);
            if (lane >= d && u > v)
                v = u;
        }
        if (lane == kWave - 1)
            scratch[w] = v;
        __syncthreads();
        int64_t m = carry, all = carry;
#pragma unroll
        for (int i = 0; i < kWavesPerBlock; ++i) {
            const int64_t x = scratch[i];
            if (i < w && x > m)
                m = x;
            if (x > all)
                all = x;
        }
        __syncthreads();
        if (m > v)
            v = m;
        if (p <= P)
            out[p] = v < n ? v : n;
        carry = all;
    }
    __syncthreads();
}

// ---- device-scope atomics used by the chained scan -------------------------
__device__ __forceinline__ uint64_t ld_agent(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void or_status(int32_t *s, int32_t bits)
{
    if (s)
        __hip_atomic_fetch_or(s, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile handled by workgroup b of n.  Workgroups are dispatched round-robin
// over the 8 XCDs (b mod 8); with MDX_XCD_SWIZZLE each XCD gets a
// contiguous run of tiles, so neighbouring tiles' partial output lines meet
// in the same L2.
#ifndef MDX_XCD_SWIZZLE
#define MDX_XCD_SWIZZLE 1
#endif
__device__ __forceinline__ int64_t tile_of_block(int64_t b, int64_t n)
{
#if MDX_XCD_SWIZZLE
    constexpr int64_t X = 8;
    const int64_t x = b % X, k = b / X, q = n / X, r = n % X;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
#else
    (void)n;
    return b;
#endif
}

// Largest q in [lo, hi) with a[q] <= x, for a non-decreasing a with
// a[lo] <= x (a has at least hi entries).
__device__ __forceinline__ int upper_index(const int64_t *a, int lo, int hi, int64_t x)
{
    int l = lo, h = hi - 1;
    while (l < h) {
        int mid = (l + h + 1) >> 1;
        if (a[mid] <= x)
            l = mid;
        else
            h = mid - 1;
    }
    return l;
}

// Range of a batch launch that holds block x: the last m in [0, M) with
// pre[m] <= x, for non-decreasing pre[0..M] with pre[0] = 0 <= x < pre[M]
// (merge m owns blocks [pre[m], pre[m+1]); merges with no blocks are
// skipped).  Called by whole waves with the same x: each round compares 64
// entries spread over the remaining range, so M <= 4096 takes two rounds.
__device__ inline int find_range(const uint32_t *pre, int M, uint32_t x)
{
    const int lane = lane_id();
    int lo = 0, span = M;  // the answer lies in [lo, lo + span)
    while (span > 1) {
        const int step = (span + kWave - 1) / kWave;
        const int off = lane * step;
        const bool ok = off < span && pre[lo + off] <= x;
        const uint64_t b = ballot(ok);  // lane 0 holds: pre[lo] <= x
        const int j = b ? 63 - __builtin_clzll(b) : 0;
        lo += j * step;
        span = step < span - j * step ? step : span - j * step;
    }
    return lo;
}

// ---- chained scan over ordered tiles (decoupled look-back) -------------------
// Status word of a tile: flag in the top 2 bits (1: its own count is
// published, 2: its inclusive prefix is published), value below.
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagIncl = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr int64_t kSpinLimit = 1ll << 24;

// Sum of the values of tiles [0, tile), run by one full wave: walks back
// from tile - 1, 64 tiles at a time, adding published counts up to the
// nearest inclusive prefix, and waits while a tile before it is still
// unpublished.  Every tile that was handed out publishes, so the wait ends;
// as a guard it gives up after kSpinLimit polls, reports
// MDX_DEV_SCAN_TIMEOUT and sets *ok = false.
__device__ inline int64_t prefix_before(const uint64_t *st, int64_t tile, int lane,
                                        int32_t *status, bool *ok)
{
    int64_t excl = 0;
    int64_t j = tile - 1;
    int64_t polls = 0;
    *ok = true;
    for (;;) {
        const int64_t idx = j - lane;
        const uint64_t s = idx >= 0 ? ld_agent(st + idx) : kFlagIncl;
        const uint64_t f = s >> 62;
        const uint64_t incl = ballot(f == 2);
        const uint64_t zero = ballot(f == 0);
        const int L = incl ? __ffsll((unsigned long long)incl) - 1 : kWave - 1;
        const uint64_t upto = (L == kWave - 1) ? ~0ull : ((2ull << L) - 1);
        if (zero & upto) {
            if (++polls > kSpinLimit) {
                if (lane == 0)
                    or_status(status, MDX_DEV_SCAN_TIMEOUT);
                *ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += wave_sum(lane <= L ? (int64_t)(s & kValMask) : 0);
        if (incl)
            break;
        j -= kWave;
    }
    return excl;
}

// Chained scan step for tile `tile` with count `agg`, run by one full wave.
// Returns the number of output rows of all earlier tiles.
__device__ inline int64_t lookback(uint64_t *st, int64_t tile, int64_t agg, int lane, int32_t *status)
{
    if (tile == 0) {
        if (lane == 0)
            st_agent(st, kFlagIncl | (uint64_t)agg);
        return 0;
    }
    if (lane == 0)
        st_agent(st + tile, kFlagAgg | (uint64_t)agg);
    bool ok;
    const int64_t excl = prefix_before(st, tile, lane, status, &ok);
    if (lane == 0)
        st_agent(st + tile, kFlagIncl | (uint64_t)(excl + agg));
    return excl;
}


}  // namespace mdx
