// Per-partition hash join (the local merge after the shuffle; arXiv
// 2101.08878, Section V-B "cuDF Merge": each worker merges the frames it
// received).  Inner equi-join, multiset semantics; left = build side.
//
// Table of partition p (see TableLayout): open addressing with linear
// probing over 16-byte slots (hash, value), split into two halves by the top
// bit of the hash so that each half has an empty marker no hash of that half
// can equal.  Hashes are stored instead of keys: fmix64 is a bijection, so
// equal hashes mean equal keys.
//
// Build (tbl_init, tbl_insert): every row claims a slot for its hash with a
// compare-and-swap; the first row of a key stores its payload in the value.
// A row that finds its hash already present marks the partition as holding
// a repeated key.  Only such partitions then run the grouped build
// (grp_reset, grp_count, grp_alloc, grp_scatter), which turns the value into
// a cursor and lays the partition's payloads out grouped by key
// ("grouped", with [gstart[s], value[s]) the group of slot s).  A key can
// hold millions of rows (a Zipf distribution's first key), so rows are
// counted and placed per workgroup first: a workgroup's rows of one slot
// meet in an LDS map and reach the slot with one global atomic, and group
// starts are allocated per chunk of slots, not per wave.
//
// Probe (probe_chain): tiles of 2048 probe rows, each inside one partition,
// are taken in order from a ticket counter.  A tile looks up its rows,
// counts its output rows, and obtains the number of output rows of all
// earlier tiles from a chained scan (each tile publishes its count, then its
// inclusive prefix; a successor sums predecessors' counts until it meets an
// inclusive prefix).  Tiles of unique-key partitions write their matches
// directly; tiles of repeated-key partitions record per-row prefixes and are
// expanded by probe_expand, which spreads a tile's output over the whole
// device in chunks (one right row can match millions of left rows).
#include <algorithm>

#include "mdx.h"
#include "mdx_internal.hpp"

namespace mdx {
namespace {

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint64_t empty_of_half(uint64_t t)
{
    return t ? 0ull : ~0ull;
}

// Slot range of partition p inside a view whose first row is o0.
__device__ __forceinline__ void part_slots(const TView &v, int64_t o0, int p, int64_t &sb,
                                           int64_t &H)
{
    const int64_t a = v.off[p], b = v.off[p + 1];
    sb = 2 * (a - o0) + 16 * (int64_t)(p - v.pb);
    H = b - a + 8;
}

// Partition of slot s: largest p in [pb, pe) with sb(p) <= s.
__device__ __forceinline__ int slot_part(const TView &v, int64_t o0, int64_t s)
{
    int l = v.pb, h = v.pe - 1;
    while (l < h) {
        const int mid = (l + h + 1) >> 1;
        if (2 * (v.off[mid] - o0) + 16 * (int64_t)(mid - v.pb) <= s)
            l = mid;
        else
            h = mid - 1;
    }
    return l;
}

// Slot of hash h in partition (sb, H), or -1.
__device__ __forceinline__ int64_t find_slot(const uint64_t *slots, int64_t sb, int64_t H,
                                             uint64_t h)
{
    const uint64_t t = h >> 63;
    const uint64_t empty = empty_of_half(t);
    const int64_t base = sb + (int64_t)t * H;
    uint64_t i = __umul64hi(h << 1, (uint64_t)H);
    for (int64_t k = 0; k < H; ++k) {
        const uint64_t w = slots[2 * (base + (int64_t)i)];
        if (w == h)
            return base + (int64_t)i;
        if (w == empty)
            return -1;
        if (++i == (uint64_t)H)
            i = 0;
    }
    return -1;
}

__device__ __forceinline__ bool skipped(const int32_t *skip)
{
    return skip && *skip != 0;
}

__device__ bool block_any_dup(const TView &v)
{
    int any = 0;
    for (int p = v.pb + (int)threadIdx.x; p < v.pe; p += kBlock)
        any |= v.flags[p];
    return __syncthreads_or(any) != 0;
}

// ---- build -----------------------------------------------------------------

// One block: the table's sanitized build offsets, cleared per-partition flags.
__device__ void table_setup_block(const int64_t *off_in, int64_t n, int64_t *off_tab,
                                  int32_t *flags, int64_t *bump, int P, int64_t *scratch)
{
    if (off_in)
        sanitize_offsets(off_in, off_tab, P, n, scratch);
    for (int p = threadIdx.x; p < P; p += kBlock) {
        flags[p] = 0;
        bump[p] = 0;
    }
}

__global__ __launch_bounds__(kBlock) void table_setup(const int64_t *__restrict__ off_in, int64_t n,
                                                      int64_t *__restrict__ off_tab,
                                                      int32_t *__restrict__ flags,
                                                      int64_t *__restrict__ bump, int P)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    table_setup_block(off_in, n, off_tab, flags, bump, P, scratch);
}

__global__ __launch_bounds__(kBlock) void tbl_init(TView v)
{
    if (skipped(v.skip))
        return;
    const int64_t o0 = v.off[v.pb];
    const int64_t total = 2 * (v.off[v.pe] - o0) + 16 * (int64_t)(v.pe - v.pb);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    u64x2 *slots = (u64x2 *)v.slots;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < total; s += stride) {
        const int p = slot_part(v, o0, s);
        int64_t sb, H;
        part_slots(v, o0, p, sb, H);
        u64x2 e;
        e.x = (s - sb < H) ? ~0ull : 0ull;
        e.y = 0;
        slots[s] = e;
    }
}

template <typename K>
__global__ __launch_bounds__(kBlock) void tbl_insert(const K *__restrict__ keys,
                                                     const int64_t *__restrict__ pay, TView v,
                                                     int32_t *status)
{
    if (skipped(v.skip))
        return;
    const int64_t o0 = v.off[v.pb], o1 = v.off[v.pe];
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t r = o0 + (int64_t)blockIdx.x * kBlock + threadIdx.x; r < o1; r += stride) {
        const uint64_t h = fmix64(key_bits(keys[r]));
        const int p = upper_index(v.off, v.pb, v.pe, r);
        if ((int)part_of(h, v.d) != p) {
            or_status(status, MDX_DEV_BAD_PARTITIONING);
            continue;
        }
        int64_t sb, H;
        part_slots(v, o0, p, sb, H);
        const uint64_t t = h >> 63;
        const uint64_t empty = empty_of_half(t);
        const int64_t base = sb + (int64_t)t * H;
        uint64_t i = __umul64hi(h << 1, (uint64_t)H);
        // The half holds at most n_p of its H = n_p + 8 slots, so an empty
        // slot exists and the walk ends within H steps.
        for (int64_t k = 0; k < H; ++k) {
            uint64_t *sp = v.slots + 2 * (base + (int64_t)i);
            uint64_t w = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (w == empty) {
                uint64_t expect = empty;
                if (__hip_atomic_compare_exchange_strong(sp, &expect, h, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)) {
                    sp[1] = (uint64_t)pay[r];
                    break;
                }
                w = expect;
            }
            if (w == h) {
                // repeated key: one store per partition suffices (a key can
                // repeat millions of times, each a store to one address)
                if (!v.flags[p])
                    v.flags[p] = 1;
                break;
            }
            if (++i == (uint64_t)H)
                i = 0;
        }
    }
}

// Repeated-key partitions: value := 0 on every slot.
__global__ __launch_bounds__(kBlock) void grp_reset(TView v)
{
    if (skipped(v.skip))
        return;
    if (!block_any_dup(v))
        return;
    const int64_t o0 = v.off[v.pb];
    const int64_t total = 2 * (v.off[v.pe] - o0) + 16 * (int64_t)(v.pe - v.pb);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < total; s += stride) {
        if (v.flags[slot_part(v, o0, s)])
            v.slots[2 * s + 1] = 0;
    }
}

// Slot of row r if r belongs to a repeated-key partition of the view, else -1.
template <typename K>
__device__ __forceinline__ int64_t dup_row_slot(const K *keys, const TView &v, int64_t o0,
                                                int64_t r, int64_t o1)
{
    if (r >= o1)
        return -1;
    const uint64_t h = fmix64(key_bits(keys[r]));
    const int p = upper_index(v.off, v.pb, v.pe, r);
    if (!v.flags[p] || (int)part_of(h, v.d) != p)
        return -1;
    int64_t sb, H;
    part_slots(v, o0, p, sb, H);
    return find_slot(v.slots, sb, H, h);
}

// ---- per-workgroup aggregation of rows by slot ------------------------------------
constexpr int kAggRows = 16384;  // rows per workgroup of grp_count / grp_scatter
constexpr int kAggMap = 2048;    // LDS map entries: slot -> rows of this workgroup
constexpr int kAggProbe = 8;     // map probes before a row goes to the slot directly
constexpr int64_t kAggNone = -1;

__device__ __forceinline__ uint32_t agg_home(int64_t s)
{
    return ((uint32_t)s * 0x9E3779B1u) >> (32 - 11);
}
static_assert(kAggMap == 1 << 11, "agg_home takes 11 bits");

// Entry of slot s in the map, inserting it if there is room within
// kAggProbe probes; -1 otherwise.  Entries are never removed, so every row of
// one slot gets the same answer.
__device__ __forceinline__ int agg_insert(int64_t *mkey, int64_t s)
{
    uint32_t h = agg_home(s);
    for (int k = 0; k < kAggProbe; ++k) {
        int64_t cur = mkey[h];
        if (cur == kAggNone) {
            cur = (int64_t)atomicCAS((unsigned long long *)&mkey[h], (unsigned long long)kAggNone,
                                     (unsigned long long)s);
            if (cur == kAggNone)
                return (int)h;
        }
        if (cur == s)
            return (int)h;
        h = (h + 1) & (kAggMap - 1);
    }
    return -1;
}

// Rows of workgroup b: [o0 + b kAggRows, ...) of the view's rows.
__device__ __forceinline__ void agg_rows(const TView &v, int64_t &o0, int64_t &r0, int64_t &r1)
{
    o0 = v.off[v.pb];
    const int64_t o1 = v.off[v.pe];
    r0 = o0 + (int64_t)blockIdx.x * kAggRows;
    r1 = r0 + kAggRows < o1 ? r0 + kAggRows : o1;
}

// value[s] += rows of the slot's key.
template <typename K>
__global__ __launch_bounds__(kBlock) void grp_count(const K *__restrict__ keys, TView v)
{
    if (skipped(v.skip))
        return;
    if (!block_any_dup(v))
        return;
    __shared__ int64_t mkey[kAggMap];
    __shared__ uint32_t mcnt[kAggMap];
    for (int i = threadIdx.x; i < kAggMap; i += kBlock) {
        mkey[i] = kAggNone;
        mcnt[i] = 0;
    }
    __syncthreads();
    int64_t o0, r0, r1;
    agg_rows(v, o0, r0, r1);
    const int64_t o1 = v.off[v.pe];
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        const int64_t s = dup_row_slot(keys, v, o0, r, o1);
        if (s < 0)
            continue;
        const int e = agg_insert(mkey, s);
        if (e >= 0)
            atomicAdd(&mcnt[e], 1u);
        else
            atomicAdd((unsigned long long *)&v.slots[2 * s + 1], 1ull);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kAggMap; i += kBlock)
        if (mkey[i] != kAggNone)
            atomicAdd((unsigned long long *)&v.slots[2 * mkey[i] + 1], (unsigned long long)mcnt[i]);
}

// Give every key of a repeated-key partition its range of the grouped array:
// gstart[s] = value[s] = (partition's first row) + running total.  Workgroup b
// takes the slots [b kAllocSlots, (b+1) kAllocSlots): per partition in it, a
// sum over its slots, one atomic on the partition's allocator, then the
// exclusive scan of its slots' counts from there.
constexpr int64_t kAllocSlots = 65536;

__device__ __forceinline__ int64_t slot_rows(const TView &v, const int64_t *slots2, int64_t s,
                                             int64_t sb, int64_t H)
{
    const uint64_t w = v.slots[2 * s];
    const uint64_t empty = empty_of_half((s - sb) >= H ? 1 : 0);
    return w == empty ? 0 : (int64_t)slots2[2 * s + 1];
}

__global__ __launch_bounds__(kBlock) void grp_alloc(TView v)
{
    if (skipped(v.skip))
        return;
    if (!block_any_dup(v))
        return;
    __shared__ int64_t scratch[kWavesPerBlock];
    __shared__ int64_t s_base;
    const int64_t o0 = v.off[v.pb];
    const int64_t total = 2 * (v.off[v.pe] - o0) + 16 * (int64_t)(v.pe - v.pb);
    const int64_t c0 = (int64_t)blockIdx.x * kAllocSlots;
    const int64_t c1 = c0 + kAllocSlots < total ? c0 + kAllocSlots : total;
    if (c0 >= c1)
        return;
    const int64_t *sv = (const int64_t *)v.slots;
    for (int p = slot_part(v, o0, c0); p < v.pe; ++p) {
        int64_t sb, H;
        part_slots(v, o0, p, sb, H);
        if (sb >= c1)
            break;
        if (!v.flags[p])
            continue;
        const int64_t a = sb > c0 ? sb : c0, e = sb + 2 * H < c1 ? sb + 2 * H : c1;
        int64_t sum = 0;
        for (int64_t x = a + threadIdx.x; x < e; x += kBlock)
            sum += slot_rows(v, sv, x, sb, H);
        int64_t all;
        (void)block_excl_scan(sum, scratch, &all);
        if (threadIdx.x == 0)
            s_base = (int64_t)atomicAdd((unsigned long long *)&v.bump[p], (unsigned long long)all);
        __syncthreads();
        int64_t carry = (v.off[p] - o0) + s_base;
        for (int64_t x0 = a; x0 < e; x0 += kBlock) {
            const int64_t x = x0 + threadIdx.x;
            const int64_t c = x < e ? slot_rows(v, sv, x, sb, H) : 0;
            int64_t tot;
            const int64_t ex = block_excl_scan(c, scratch, &tot);
            if (x < e && c > 0) {
                v.gstart[x] = carry + ex;
                v.slots[2 * x + 1] = (uint64_t)(carry + ex);
            }
            carry += tot;
        }
        __syncthreads();  // s_base is reused by the next partition
    }
}

// grouped[value[s]++] = payload, for every row of a repeated-key partition.
// First the workgroup counts its rows per slot in the map and reserves one
// range per slot; then every row takes the next place of its slot's range
// (rows the map could not hold take a place from the slot directly).
template <typename K>
__global__ __launch_bounds__(kBlock) void grp_scatter(const K *__restrict__ keys,
                                                      const int64_t *__restrict__ pay, TView v)
{
    if (skipped(v.skip))
        return;
    if (!block_any_dup(v))
        return;
    __shared__ int64_t mkey[kAggMap];
    __shared__ int64_t mbase[kAggMap];
    __shared__ uint32_t mcnt[kAggMap];
    // every row's map entry from the first pass: kRowSkip (no repeated-key
    // row), kRowDirect (not in the map: takes its place from the slot), or
    // the entry
    constexpr int16_t kRowSkip = -2, kRowDirect = -1;
    __shared__ int16_t rent[kAggRows];
    for (int i = threadIdx.x; i < kAggMap; i += kBlock) {
        mkey[i] = kAggNone;
        mcnt[i] = 0;
    }
    __syncthreads();
    int64_t o0, r0, r1;
    agg_rows(v, o0, r0, r1);
    const int64_t o1 = v.off[v.pe];
    for (int i = threadIdx.x; i < kAggRows; i += kBlock) {
        const int64_t r = r0 + i;
        const int64_t s = dup_row_slot(keys, v, o0, r, o1);
        int e = kRowSkip;
        if (s >= 0) {
            e = agg_insert(mkey, s);
            if (e >= 0)
                atomicAdd(&mcnt[e], 1u);
            else
                e = kRowDirect;
        }
        rent[i] = (int16_t)e;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kAggMap; i += kBlock) {
        if (mkey[i] != kAggNone)
            mbase[i] = (int64_t)atomicAdd((unsigned long long *)&v.slots[2 * mkey[i] + 1],
                                          (unsigned long long)mcnt[i]);
        mcnt[i] = 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kAggRows; i += kBlock) {
        const int e = rent[i];
        if (e == kRowSkip)
            continue;
        const int64_t r = r0 + i;
        int64_t at;
        if (e >= 0) {
            at = mbase[e] + (int64_t)atomicAdd(&mcnt[e], 1u);
        } else {
            const int64_t s = dup_row_slot(keys, v, o0, r, o1);
            at = (int64_t)atomicAdd((unsigned long long *)&v.slots[2 * s + 1], 1ull);
        }
        v.grouped[at] = pay[r];
    }
}

// ---- probe -----------------------------------------------------------------

// Block 0 plans the probe tiles; every block clears its share of the
// chained-scan status.
__device__ void probe_plan_blocks(const int64_t *offR, int64_t n, int P, const ProbeWs &w,
                                  int64_t *scratch)
{
    if (blockIdx.x == 0) {
        sanitize_offsets(offR, w.off, P, n, scratch);
        int64_t carry = 0;
        for (int base = 0; base < P; base += kBlock) {
            const int p = base + threadIdx.x;
            const int64_t nt =
                p < P ? (w.off[p + 1] - w.off[p] + kProbeTile - 1) / kProbeTile : 0;
            int64_t tot;
            const int64_t ex = block_excl_scan(nt, scratch, &tot);
            if (p < P) {
                w.tile_start[p] = carry + ex;
                w.ticket[p] = 0;
            }
            carry += tot;
        }
        if (threadIdx.x == 0) {
            w.tile_start[P] = carry;
            *w.ndefer = 0;
        }
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < w.max_tiles; i += stride)
        w.status[i] = 0;
}

__global__ __launch_bounds__(kBlock) void probe_plan(const int64_t *__restrict__ offR, int64_t n,
                                                     int P, ProbeWs w, const int32_t *skip)
{
    if (skipped(skip))
        return;
    __shared__ int64_t scratch[kWavesPerBlock];
    probe_plan_blocks(offR, n, P, w, scratch);
}

// Set-up of a merge's global-table join in one block: per-partition build
// and probe offsets taken from the first-pass offsets (every stride-th
// entry), the table's offsets and flags, the probe plan.
__global__ __launch_bounds__(kBlock) void fallback_setup(
    const int64_t *__restrict__ offAL, const int64_t *__restrict__ offAR, int stride, int P,
    int64_t n_build, int64_t n_probe, int64_t *offPL, int64_t *offPR, int64_t *off_tab,
    int32_t *flags, int64_t *bump, ProbeWs w, const int32_t *skip)
{
    if (skipped(skip))
        return;
    __shared__ int64_t scratch[kWavesPerBlock];
    for (int p = threadIdx.x; p <= P; p += kBlock) {
        offPL[p] = offAL[(int64_t)p * stride];
        offPR[p] = offAR[(int64_t)p * stride];
    }
    __syncthreads();
    table_setup_block(offPL, n_build, off_tab, flags, bump, P, scratch);
    probe_plan_blocks(offPR, n_probe, P, w, scratch);
}

template <typename K>
__global__ __launch_bounds__(kBlock) void probe_chain(const K *__restrict__ pk,
                                                      const int64_t *__restrict__ pv, TView v,
                                                      int group, ProbeWs w, ProbeOut o,
                                                      int32_t *status)
{
    if (skipped(v.skip))
        return;
    constexpr int RP = kProbeRows;
    __shared__ int64_t s_tile, s_excl;
    __shared__ int64_t cw[RP][kWavesPerBlock];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int64_t t_begin = w.tile_start[v.pb], t_end = w.tile_start[v.pe];
    const int64_t o0 = v.off[v.pb];
    K *out_key = (K *)o.key;

    for (;;) {
        if (tid == 0)
            s_tile = t_begin + (int64_t)atomicAdd(&w.ticket[group], 1u);
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= t_end)
            break;
        const int p = upper_index(w.tile_start, v.pb, v.pe, tile);
        const int64_t rbeg = w.off[p] + (tile - w.tile_start[p]) * kProbeTile;
        const int64_t rlim = w.off[p + 1];
        const int64_t rend = rbeg + kProbeTile < rlim ? rbeg + kProbeTile : rlim;
        const bool dup = v.flags[p] != 0;
        int64_t sb, H;
        part_slots(v, o0, p, sb, H);

        K kk[RP];
        int64_t vv[RP], m[RP], lv[RP];
        bool bad = false;
#pragma unroll
        for (int c = 0; c < RP; ++c) {
            const int64_t r = rbeg + (int64_t)c * kBlock + tid;
            const bool valid = r < rend;
            kk[c] = valid ? __builtin_nontemporal_load(pk + r) : K(0);
            vv[c] = valid ? __builtin_nontemporal_load(pv + r) : 0;
        }
#pragma unroll
        for (int c = 0; c < RP; ++c) {
            const int64_t r = rbeg + (int64_t)c * kBlock + tid;
            m[c] = 0;
            lv[c] = 0;
            if (r < rend) {
                const uint64_t h = fmix64(key_bits(kk[c]));
                if ((int)part_of(h, v.d) != p) {
                    bad = true;
                } else {
                    const int64_t s = find_slot(v.slots, sb, H, h);
                    if (s >= 0) {
                        const uint64_t val = v.slots[2 * s + 1];
                        if (!dup) {
                            m[c] = 1;
                            lv[c] = (int64_t)val;
                        } else {
                            const int64_t g0 = v.gstart[s];
                            m[c] = (int64_t)val - g0;
                            lv[c] = g0;
                        }
                    }
                }
            }
        }
        if (bad)
            or_status(status, MDX_DEV_BAD_PARTITIONING);

        // Output rank of every row: order (c, thread), i.e. row order.
        int64_t mex[RP];
#pragma unroll
        for (int c = 0; c < RP; ++c) {
            const int64_t inc = wave_incl_scan(m[c], lane);
            mex[c] = inc - m[c];
            if (lane == kWave - 1)
                cw[c][wv] = inc;
        }
        __syncthreads();
        int64_t run = 0, cbase[RP];
#pragma unroll
        for (int c = 0; c < RP; ++c) {
#pragma unroll
            for (int ww = 0; ww < kWavesPerBlock; ++ww) {
                const int64_t x = cw[c][ww];
                if (ww == wv)
                    cbase[c] = run;
                run += x;
            }
        }
        const int64_t M = run;
        if (wv == 0) {
            const int64_t ex = lookback(w.status, tile, M, lane, status);
            if (lane == 0) {
                s_excl = ex;
                w.tile_base[tile] = ex;
            }
        }
        __syncthreads();
        const int64_t E = s_excl;
        if (E + M > o.cap) {
            if (tid == 0 && M > 0)
                or_status(status, MDX_DEV_OUTPUT_OVERFLOW);
        } else if (!dup) {
#pragma unroll
            for (int c = 0; c < RP; ++c) {
                if (m[c]) {
                    const int64_t at = E + cbase[c] + mex[c];
                    out_key[at] = kk[c];
                    o.lpay[at] = lv[c];
                    o.rpay[at] = vv[c];
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < RP; ++c) {
                const int64_t r = rbeg + (int64_t)c * kBlock + tid;
                if (r < rend) {
                    w.row_pre[r] = cbase[c] + mex[c];
                    w.row_gs[r] = lv[c];
                }
            }
            if (tid == 0 && M > 0) {
                const uint32_t d = atomicAdd(w.ndefer, 1u);
                Deferred D;
                D.rbeg = rbeg;
                D.rend = rend;
                D.base = E;
                D.count = M;
                D.group = group;
                w.defer[d] = D;
            }
        }
        __syncthreads();
    }
}

template <typename K>
__global__ __launch_bounds__(kBlock) void probe_expand(const K *__restrict__ pk,
                                                       const int64_t *__restrict__ pv, TView v,
                                                       int group, ProbeWs w, ProbeOut o)
{
    if (skipped(v.skip))
        return;
    constexpr int64_t CH = 4096;  // output rows per chunk
    __shared__ int64_t pre[kProbeTile];
    const uint32_t nd = *w.ndefer;
    const int64_t G = gridDim.x;
    K *out_key = (K *)o.key;
    int64_t acc = 0;  // global index of the current entry's first chunk
    for (uint32_t e = 0; e < nd; ++e) {
        const Deferred D = w.defer[e];
        if (D.group != group)
            continue;
        const int64_t nch = (D.count + CH - 1) / CH;
        int64_t j = (((int64_t)blockIdx.x - acc) % G + G) % G;
        if (j < nch) {
            const int rows = (int)(D.rend - D.rbeg);
            for (int i = threadIdx.x; i < rows; i += kBlock)
                pre[i] = w.row_pre[D.rbeg + i];
            __syncthreads();
            for (; j < nch; j += G) {
                const int64_t lim = (j + 1) * CH < D.count ? (j + 1) * CH : D.count;
                for (int64_t q = j * CH + threadIdx.x; q < lim; q += kBlock) {
                    int l = 0, h = rows - 1;  // last row whose prefix <= q
                    while (l < h) {
                        const int mid = (l + h + 1) >> 1;
                        if (pre[mid] <= q)
                            l = mid;
                        else
                            h = mid - 1;
                    }
                    const int64_t r = D.rbeg + l;
                    const int64_t at = D.base + q;
                    out_key[at] = pk[r];
                    o.lpay[at] = v.grouped[w.row_gs[r] + (q - pre[l])];
                    o.rpay[at] = pv[r];
                }
            }
            __syncthreads();
        }
        acc += nch;
    }
}

__global__ __launch_bounds__(kBlock) void probe_finalize(int P, ProbeWs w, ProbeOut o,
                                                         const int32_t *skip)
{
    if (skipped(skip))
        return;
    const int64_t TT = w.tile_start[P];
    const int64_t total = TT > 0 ? (int64_t)(ld_agent(w.status + TT - 1) & kValMask) : 0;
    for (int p = threadIdx.x; p <= P; p += kBlock) {
        const int64_t t = w.tile_start[p];
        o.offsets[p] = t < TT ? w.tile_base[t] : total;
    }
}

// ---- count-only join --------------------------------------------------------------
// The table of the build side holds, per distinct hash, the number of build
// rows with that hash (slot value; tbl_init sets it to 0).  Both sides'
// rows are first counted per workgroup in an LDS map of hashes, so a key
// repeated millions of times costs one global update per workgroup; rows
// the map cannot take go to the table one by one.
constexpr int kCountRows = 8;  // rows per thread loaded together
#ifndef MDX_COUNT_MAP_BITS
#define MDX_COUNT_MAP_BITS 12
#endif
#ifndef MDX_COUNT_WG_ROWS
#define MDX_COUNT_WG_ROWS 16384
#endif
// On 5E7 x 5E7 Zipf(1.1) keys (P = 16) the count took 2.07 ms with 2048
// entries, 1.98 with 4096 and 2.83 with 8192 (96 KB of LDS: fewer
// workgroups per CU); 8192 or 32768 rows per workgroup instead of 16384
// were slower.
constexpr int kCountMapBits = MDX_COUNT_MAP_BITS;
constexpr int kCountMap = 1 << kCountMapBits;  // LDS map entries
constexpr int kCountWgRows = MDX_COUNT_WG_ROWS;  // rows per workgroup

// Entry of hash h in the LDS map (inserted if there is room within
// kAggProbe probes), or -1.  ~0 marks an empty entry, so a row whose hash is
// ~0 is never mapped.
__device__ __forceinline__ int hmap_insert(uint64_t *mkey, uint64_t h)
{
    if (h == ~0ull)
        return -1;
    // bits from 32 up: the partition takes the low bits, a slot's home the top ones
    uint32_t i = (uint32_t)(h >> 32) >> (32 - kCountMapBits);
    for (int k = 0; k < kAggProbe; ++k) {
        uint64_t cur = mkey[i];
        if (cur == ~0ull) {
            cur = atomicCAS((unsigned long long *)&mkey[i], ~0ull, (unsigned long long)h);
            if (cur == ~0ull)
                return (int)i;
        }
        if (cur == h)
            return (int)i;
        i = (i + 1) & (kCountMap - 1);
    }
    return -1;
}

// value[slot of h] += c in partition p, claiming the slot if h is new.  The
// half holds at most n_p distinct hashes in its H = n_p + 8 slots.
__device__ __forceinline__ void slot_add(const TView &v, int64_t o0, int p, uint64_t h,
                                         uint64_t c)
{
    int64_t sb, H;
    part_slots(v, o0, p, sb, H);
    const uint64_t t = h >> 63;
    const uint64_t empty = empty_of_half(t);
    const int64_t base = sb + (int64_t)t * H;
    uint64_t i = __umul64hi(h << 1, (uint64_t)H);
    for (int64_t k = 0; k < H; ++k) {
        uint64_t *sp = v.slots + 2 * (base + (int64_t)i);
        uint64_t w = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (w == empty) {
            uint64_t expect = empty;
            if (__hip_atomic_compare_exchange_strong(sp, &expect, h, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                atomicAdd((unsigned long long *)(sp + 1), (unsigned long long)c);
                return;
            }
            w = expect;
        }
        if (w == h) {
            atomicAdd((unsigned long long *)(sp + 1), (unsigned long long)c);
            return;
        }
        if (++i == (uint64_t)H)
            i = 0;
    }
}

// Rows [r0, r1) of the workgroup's share (kCountWgRows rows each), kCountRows per
// thread loaded together; fn(row, hash, partition) for every row in its
// partition, the others reported.
template <typename K, typename Fn>
__device__ __forceinline__ void count_rows(const K *__restrict__ keys, const int64_t *off, int P,
                                           const Dest &d, int64_t r0, int64_t r1, int32_t *status,
                                           Fn fn)
{
    bool bad = false;
    for (int64_t b = r0; b < r1; b += (int64_t)kCountRows * kBlock) {
        K k[kCountRows];
#pragma unroll
        for (int j = 0; j < kCountRows; ++j) {
            const int64_t r = b + (int64_t)j * kBlock + threadIdx.x;
            k[j] = r < r1 ? __builtin_nontemporal_load(keys + r) : K(0);
        }
#pragma unroll
        for (int j = 0; j < kCountRows; ++j) {
            const int64_t r = b + (int64_t)j * kBlock + threadIdx.x;
            if (r < r1) {
                const uint64_t h = fmix64(key_bits(k[j]));
                const int p = upper_index(off, 0, P, r);
                if ((int)part_of(h, d) != p)
                    bad = true;
                else
                    fn(h, p);
            }
        }
    }
    if (bad)
        or_status(status, MDX_DEV_BAD_PARTITIONING);
}

// Block: the sanitized build offsets into the table, the sanitized probe
// offsets, per-partition counts cleared.
__global__ __launch_bounds__(kBlock) void cnt_setup(const int64_t *__restrict__ lofs,
                                                    int64_t n_build,
                                                    const int64_t *__restrict__ rofs,
                                                    int64_t n_probe, int64_t *off_tab,
                                                    int64_t *off_probe, uint64_t *pcount, int P)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    sanitize_offsets(lofs, off_tab, P, n_build, scratch);
    sanitize_offsets(rofs, off_probe, P, n_probe, scratch);
    for (int p = threadIdx.x; p < P; p += kBlock)
        pcount[p] = 0;
}

template <typename K>
__global__ __launch_bounds__(kBlock) void cnt_insert(const K *__restrict__ keys, TView v,
                                                     int32_t *status)
{
    __shared__ uint64_t mkey[kCountMap];
    __shared__ uint32_t mcnt[kCountMap];
    for (int i = threadIdx.x; i < kCountMap; i += kBlock) {
        mkey[i] = ~0ull;
        mcnt[i] = 0;
    }
    __syncthreads();
    const int64_t o0 = v.off[0], o1 = v.off[v.pe];
    const int64_t r0 = o0 + (int64_t)blockIdx.x * kCountWgRows;
    const int64_t r1 = r0 + kCountWgRows < o1 ? r0 + kCountWgRows : o1;
    count_rows(keys, v.off, v.pe, v.d, r0, r1, status, [&](uint64_t h, int p) {
        const int e = hmap_insert(mkey, h);
        if (e >= 0)
            atomicAdd(&mcnt[e], 1u);
        else
            slot_add(v, o0, p, h, 1);
    });
    __syncthreads();
    for (int i = threadIdx.x; i < kCountMap; i += kBlock)
        if (mkey[i] != ~0ull)
            slot_add(v, o0, (int)part_of(mkey[i], v.d), mkey[i], mcnt[i]);
}

// Build rows of hash h in partition p (0 when absent).
__device__ __forceinline__ uint64_t slot_count(const TView &v, int64_t o0, int p, uint64_t h)
{
    int64_t sb, H;
    part_slots(v, o0, p, sb, H);
    const int64_t s = find_slot(v.slots, sb, H, h);
    return s >= 0 ? v.slots[2 * s + 1] : 0;
}

template <typename K>
__global__ __launch_bounds__(kBlock) void cnt_probe(const K *__restrict__ keys,
                                                    const int64_t *__restrict__ off_probe,
                                                    TView v, uint64_t *pcount, int32_t *status)
{
    extern __shared__ unsigned long long psum[];  // [P]
    __shared__ uint64_t mkey[kCountMap];
    __shared__ uint32_t mcnt[kCountMap];
    const int P = v.pe;
    for (int i = threadIdx.x; i < kCountMap; i += kBlock) {
        mkey[i] = ~0ull;
        mcnt[i] = 0;
    }
    for (int p = threadIdx.x; p < P; p += kBlock)
        psum[p] = 0;
    __syncthreads();
    const int64_t o0 = v.off[0];
    const int64_t n = off_probe[P];
    const int64_t r0 = off_probe[0] + (int64_t)blockIdx.x * kCountWgRows;
    const int64_t r1 = r0 + kCountWgRows < n ? r0 + kCountWgRows : n;
    count_rows(keys, off_probe, P, v.d, r0, r1, status, [&](uint64_t h, int p) {
        const int e = hmap_insert(mkey, h);
        if (e >= 0) {
            atomicAdd(&mcnt[e], 1u);
        } else {
            const uint64_t c = slot_count(v, o0, p, h);
            if (c)
                atomicAdd(&psum[p], (unsigned long long)c);
        }
    });
    __syncthreads();
    for (int i = threadIdx.x; i < kCountMap; i += kBlock) {
        const uint64_t h = mkey[i];
        if (h != ~0ull) {
            const int p = (int)part_of(h, v.d);
            const uint64_t c = slot_count(v, o0, p, h);
            if (c)
                atomicAdd(&psum[p], (unsigned long long)(c * mcnt[i]));
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += kBlock)
        if (psum[p])
            atomicAdd((unsigned long long *)&pcount[p], psum[p]);
}

// Block: out_offsets = exclusive prefix of the per-partition counts.
__global__ __launch_bounds__(kBlock) void cnt_finalize(const uint64_t *__restrict__ pcount, int P,
                                                       int64_t *out_offsets)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    int64_t carry = 0;
    for (int base = 0; base < P; base += kBlock) {
        const int p = base + threadIdx.x;
        const int64_t c = p < P ? (int64_t)pcount[p] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(c, scratch, &tot);
        if (p < P)
            out_offsets[p] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0)
        out_offsets[P] = carry;
}

// Workgroups of the grid-stride build and probe kernels: a full device, or
// fewer when the caller sizes the grid to its rows (max_blocks > 0).
static int table_grid(int max_blocks)
{
    const int full = device_fill_blocks();
    return max_blocks > 0 && max_blocks < full ? max_blocks : full;
}

template <typename K>
hipError_t run_build(const K *keys, const int64_t *pay, const TView &v, int64_t rows,
                     int32_t *status, int max_blocks, hipStream_t s)
{
    const int G = table_grid(max_blocks);
    // the grouping kernels' workgroups each take a fixed share of the rows
    // (of the slots: 2 rows + 16 P)
    const int64_t P = v.pe - v.pb;
    const unsigned Gr = (unsigned)std::max<int64_t>(1, (rows + kAggRows - 1) / kAggRows);
    const unsigned Gs = (unsigned)std::max<int64_t>(1, (2 * rows + 16 * P + kAllocSlots - 1) /
                                                           kAllocSlots);
    trace_begin("tbl_init", s);
    hipLaunchKernelGGL(tbl_init, dim3(G), dim3(kBlock), 0, s, v);
    trace_end("tbl_init", s);
    trace_begin("tbl_insert", s);
    hipLaunchKernelGGL((tbl_insert<K>), dim3(G), dim3(kBlock), 0, s, keys, pay, v, status);
    trace_end("tbl_insert", s);
    hipLaunchKernelGGL(grp_reset, dim3(G), dim3(kBlock), 0, s, v);
    trace_begin("grp_count", s);
    hipLaunchKernelGGL((grp_count<K>), dim3(Gr), dim3(kBlock), 0, s, keys, v);
    trace_end("grp_count", s);
    trace_begin("grp_alloc", s);
    hipLaunchKernelGGL(grp_alloc, dim3(Gs), dim3(kBlock), 0, s, v);
    trace_end("grp_alloc", s);
    trace_begin("grp_scatter", s);
    hipLaunchKernelGGL((grp_scatter<K>), dim3(Gr), dim3(kBlock), 0, s, keys, pay, v);
    trace_end("grp_scatter", s);
    return hipGetLastError();
}

template <typename K>
hipError_t run_probe_group(const K *pk, const int64_t *pv, const TView &v, int group,
                           const ProbeWs &w, const ProbeOut &o, int32_t *status, int max_blocks,
                           hipStream_t s)
{
    const int G = table_grid(max_blocks);
    trace_begin("probe_chain", s);
    hipLaunchKernelGGL((probe_chain<K>), dim3(G), dim3(kBlock), 0, s, pk, pv, v, group, w, o,
                       status);
    trace_end("probe_chain", s);
    // The expansion's work is the output rows, which can be millions for one
    // probe row: it always gets a full device (it returns at once when no
    // tile deferred rows).
    trace_begin("probe_expand", s);
    hipLaunchKernelGGL((probe_expand<K>), dim3(table_grid(0)), dim3(kBlock), 0, s, pk, pv, v,
                       group, w, o);
    trace_end("probe_expand", s);
    return hipGetLastError();
}

template <typename K>
hipError_t run_count(const K *lk, const int64_t *lofs, int64_t n_build, const K *rk,
                     const int64_t *rofs, int64_t n_probe, const TView &v, int64_t *off_probe,
                     uint64_t *pcount, int64_t *out_offsets, int32_t *status, hipStream_t s)
{
    const int P = v.pe;
    hipLaunchKernelGGL(cnt_setup, dim3(1), dim3(kBlock), 0, s, lofs, n_build, rofs, n_probe,
                       (int64_t *)v.off, off_probe, pcount, P);
    trace_begin("tbl_init", s);
    hipLaunchKernelGGL(tbl_init, dim3(table_grid(0)), dim3(kBlock), 0, s, v);
    trace_end("tbl_init", s);
    if (n_build > 0) {
        trace_begin("cnt_insert", s);
        hipLaunchKernelGGL((cnt_insert<K>),
                           dim3((unsigned)((n_build + kCountWgRows - 1) / kCountWgRows)),
                           dim3(kBlock), 0, s, lk, v, status);
        trace_end("cnt_insert", s);
    }
    if (n_probe > 0) {
        trace_begin("cnt_probe", s);
        hipLaunchKernelGGL((cnt_probe<K>),
                           dim3((unsigned)((n_probe + kCountWgRows - 1) / kCountWgRows)),
                           dim3(kBlock), (size_t)P * 8, s, rk, off_probe, v, pcount, status);
        trace_end("cnt_probe", s);
    }
    hipLaunchKernelGGL(cnt_finalize, dim3(1), dim3(kBlock), 0, s, pcount, P, out_offsets);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_join_count(const void *lk, const int64_t *lofs, int64_t n_build, const void *rk,
                             const int64_t *rofs, int64_t n_probe, int key_bytes, const TView &v,
                             int64_t *off_probe, uint64_t *pcount, int64_t *out_offsets,
                             int32_t *status, hipStream_t s)
{
    if (key_bytes == 8)
        return run_count<int64_t>((const int64_t *)lk, lofs, n_build, (const int64_t *)rk, rofs,
                                  n_probe, v, off_probe, pcount, out_offsets, status, s);
    return run_count<int32_t>((const int32_t *)lk, lofs, n_build, (const int32_t *)rk, rofs,
                              n_probe, v, off_probe, pcount, out_offsets, status, s);
}

hipError_t launch_table_setup(const int64_t *off_in, int64_t n, int64_t *off_tab, int32_t *flags,
                              int64_t *bump, int32_t P, hipStream_t s)
{
    hipLaunchKernelGGL(table_setup, dim3(1), dim3(kBlock), 0, s, off_in, n, off_tab, flags, bump,
                       P);
    return hipGetLastError();
}

hipError_t launch_build(const void *keys, const int64_t *pay, int key_bytes, const TView &v,
                        int64_t rows, int32_t *status, int max_blocks, hipStream_t s)
{
    if (key_bytes == 8)
        return run_build<int64_t>((const int64_t *)keys, pay, v, rows, status, max_blocks, s);
    return run_build<int32_t>((const int32_t *)keys, pay, v, rows, status, max_blocks, s);
}

hipError_t launch_fallback_setup(const int64_t *offAL, const int64_t *offAR, int stride,
                                 int32_t P, int64_t n_build, int64_t n_probe, int64_t *offPL,
                                 int64_t *offPR, int64_t *off_tab, int32_t *flags, int64_t *bump,
                                 const ProbeWs &w, const int32_t *skip, hipStream_t s)
{
    hipLaunchKernelGGL(fallback_setup, dim3(1), dim3(kBlock), 0, s, offAL, offAR, stride, P,
                       n_build, n_probe, offPL, offPR, off_tab, flags, bump, w, skip);
    return hipGetLastError();
}

hipError_t launch_probe_plan(const int64_t *offR, int64_t n, int32_t P, const ProbeWs &w,
                             const int32_t *skip, hipStream_t s)
{
    const int G = device_fill_blocks() / 4 > 0 ? device_fill_blocks() / 4 : 1;
    hipLaunchKernelGGL(probe_plan, dim3(G), dim3(kBlock), 0, s, offR, n, P, w, skip);
    return hipGetLastError();
}

hipError_t launch_probe_group(const void *pkeys, const int64_t *ppay, int key_bytes, int32_t P,
                              const TView &v, int group, const ProbeWs &w, const ProbeOut &o,
                              int32_t *status, int max_blocks, hipStream_t s)
{
    (void)P;
    if (key_bytes == 8)
        return run_probe_group<int64_t>((const int64_t *)pkeys, ppay, v, group, w, o, status,
                                        max_blocks, s);
    return run_probe_group<int32_t>((const int32_t *)pkeys, ppay, v, group, w, o, status,
                                    max_blocks, s);
}

hipError_t launch_probe_finalize(int32_t P, const ProbeWs &w, const ProbeOut &o,
                                 const int32_t *skip, hipStream_t s)
{
    hipLaunchKernelGGL(probe_finalize, dim3(1), dim3(kBlock), 0, s, P, w, o, skip);
    return hipGetLastError();
}

}  // namespace mdx
