// Stable hash partition of one table into P packed destination buffers.
//
// The shuffle's local half (arXiv 2101.08878, Section V-B, cuDF merge with
// "Shuffle: True"): each row goes to destination p = fmix64(key) mod P, and
// destination p's rows are packed, in input order, into [off[p], off[p+1]).
//
// Three passes over tiles of T = kBlock * R rows (512 x 8 = 4096):
//   part_hist       keys only: per-tile counts per destination (LDS atomics;
//                   a wave's ballots when there are at most 4 destinations)
//   part_scan_tiles per destination, exclusive prefix over tiles (in place)
//   part_offsets    exclusive prefix over destinations -> off[0..P]
//   part_scatter    keys + payloads: rank rows inside the tile with wave
//                   ballots (one ballot per bit of p gives every lane the
//                   mask of lanes with its destination; mbcnt of that mask is
//                   its rank among them), stage the tile in LDS sorted by
//                   destination, then write every destination's run with
//                   consecutive lanes on consecutive addresses.
// A row's output position is off[p] + (rows of p in earlier tiles) + (rows
// of p earlier in this tile), which is the stable counting-sort position.
//
// A merge runs each step once for its two tables, and splits every bucket
// again with the segmented pass below (seg_*), whose histogram counts digit
// bytes the first scatter wrote beside its rows.
#include <string.h>

#include "mdx_internal.hpp"

namespace mdx {
namespace {

// ---- one or two tables per launch -------------------------------------------
// A merge partitions its build and probe tables with the same destinations,
// so each step runs once for both: per-tile grids cover the first table's
// tiles, then the second's (the XCD-contiguous order runs over the combined
// range); per-destination and per-segment grids take one block range per
// table.  A single table is the pair with an empty second table.
template <typename K>
struct PartTable {
    const K *keys;
    const int64_t *pay;
    int64_t n, ntiles;
    K *keys_out;
    int64_t *pay_out;
    int64_t *off;     // [D + 1]
    uint8_t *dig;     // optional: one digit byte per output row
    int64_t *cnt;     // [D][ntiles]: counts, then exclusive prefixes
    int64_t *totals;  // [D]
};

template <typename K>
struct PartPair {
    PartTable<K> t[2];
};

// Table `second` of a pair, by field-wise selects on the kernel arguments.
template <typename K>
__device__ __forceinline__ PartTable<K> pick(const PartPair<K> &T, bool second)
{
    const PartTable<K> &a = T.t[0], &b = T.t[1];
    PartTable<K> r;
    r.keys = second ? b.keys : a.keys;
    r.pay = second ? b.pay : a.pay;
    r.n = second ? b.n : a.n;
    r.ntiles = second ? b.ntiles : a.ntiles;
    r.keys_out = second ? b.keys_out : a.keys_out;
    r.pay_out = second ? b.pay_out : a.pay_out;
    r.off = second ? b.off : a.off;
    r.dig = second ? b.dig : a.dig;
    r.cnt = second ? b.cnt : a.cnt;
    r.totals = second ? b.totals : a.totals;
    return r;
}

// Histograms of at most this many destinations count by ballot: a whole
// wave's LDS atomics on a few addresses serialize.
constexpr int kFewDest = 4;

// Counts of tile `tile` of table tb per destination into tb.cnt.  FEW: the
// destinations may be few enough to count by ballot.
template <typename K, int R, bool FEW>
__device__ __forceinline__ void hist_tile(const PartTable<K> &tb, int64_t tile, const Dest &d,
                                          uint32_t *hist)
{
    const int tid = threadIdx.x;
    const int P = d.ndest;  // destinations
    for (int p = tid; p < P; p += kBlock)
        hist[p] = 0;
    const int64_t row0 = tile * (int64_t)(kBlock * R);
    const bool few = FEW && P <= kFewDest;
    uint32_t wc[kFewDest] = {};  // with few destinations: the wave's counts
    auto count = [&](bool valid, uint32_t p) {
        if (few) {
#pragma unroll
            for (int q = 0; q < kFewDest; ++q)
                if (q < P)
                    wc[q] += (uint32_t)__popcll(ballot(valid && p == (uint32_t)q));
        } else if (valid) {
            atomicAdd(&hist[p], 1u);
        }
    };
    // Keys are read 16 bytes per lane when the column is 16-byte aligned
    // (the counts do not depend on which thread reads which row).
    constexpr int V = 16 / (int)sizeof(K);  // keys per 16-byte load
    if (R % V == 0 && ((uintptr_t)tb.keys & 15) == 0) {
        // Thread tid, load j: rows row0 + (j kBlock + tid) V + [0, V).
        typedef K KV __attribute__((ext_vector_type(V)));
        K k[R];
#pragma unroll
        for (int j = 0; j < R / V; ++j) {
            const int64_t r = row0 + ((int64_t)j * kBlock + tid) * V;
            if (r + V <= tb.n) {
                const KV x = __builtin_nontemporal_load((const KV *)(tb.keys + r));
#pragma unroll
                for (int v = 0; v < V; ++v)
                    k[j * V + v] = x[v];
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    k[j * V + v] = r + v < tb.n ? tb.keys[r + v] : K(0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < R / V; ++j) {
            const int64_t r = row0 + ((int64_t)j * kBlock + tid) * V;
#pragma unroll
            for (int v = 0; v < V; ++v)
                count(r + v < tb.n, dest_of(fmix64(key_bits(k[j * V + v])), d));
        }
    } else {
        K k[R];
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int64_t r = row0 + (int64_t)c * kBlock + tid;
            k[c] = r < tb.n ? __builtin_nontemporal_load(tb.keys + r) : K(0);
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int64_t r = row0 + (int64_t)c * kBlock + tid;
            count(r < tb.n, dest_of(fmix64(key_bits(k[c])), d));
        }
    }
    if (few && (tid & (kWave - 1)) == 0) {
#pragma unroll
        for (int q = 0; q < kFewDest; ++q)
            if (q < P && wc[q] != 0)
                atomicAdd(&hist[q], wc[q]);
    }
    __syncthreads();
    for (int p = tid; p < P; p += kBlock)
        tb.cnt[(int64_t)p * tb.ntiles + tile] = hist[p];
}

template <typename K, int R, bool FEW>
__global__ __launch_bounds__(kBlock) void part_hist(PartPair<K> T, Dest d)
{
    extern __shared__ uint32_t hist[];
    // XCD-contiguous tile order: the counts of neighbouring tiles share cache
    // lines, which then fill in one L2
    const int64_t g = tile_of_block(blockIdx.x, gridDim.x);
    const bool second = g >= T.t[0].ntiles;
    hist_tile<K, R, FEW>(pick(T, second), second ? g - T.t[0].ntiles : g, d, hist);
}

// Block p: exclusive prefix of cnt[p][0..ntiles) in place, total to totals[p].
// Rounds of kBlock * kScanV counts: loaded and stored with consecutive lanes
// on consecutive counts, staged in LDS so that thread t sums the kScanV
// consecutive counts [t kScanV, (t+1) kScanV) (rows padded by one count, so
// those reads spread over the banks), then one block scan of the sums.
constexpr int kScanV = 16;
constexpr int kScanChunk = kBlock * kScanV;

__device__ __forceinline__ int scan_slot(int e)
{
    return e + e / kScanV;
}

// Destination p of one table: prefix of its row of counts, total to totals[p].
__device__ __forceinline__ void scan_tiles_of(int64_t *cnt, int64_t ntiles, int64_t *totals, int p)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    __shared__ int64_t buf[kScanChunk + kBlock];
    const int tid = threadIdx.x;
    int64_t *row = cnt + (int64_t)p * ntiles;
    int64_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += kScanChunk) {
        const int m = (int)(ntiles - base < kScanChunk ? ntiles - base : kScanChunk);
#pragma unroll
        for (int j = 0; j < kScanV; ++j) {
            const int e = j * kBlock + tid;
            buf[scan_slot(e)] = e < m ? row[base + e] : 0;
        }
        __syncthreads();
        int64_t v[kScanV], sum = 0;
#pragma unroll
        for (int i = 0; i < kScanV; ++i) {
            v[i] = buf[scan_slot(tid * kScanV + i)];
            sum += v[i];
        }
        int64_t tot;
        int64_t run = carry + block_excl_scan(sum, scratch, &tot);
#pragma unroll
        for (int i = 0; i < kScanV; ++i) {
            buf[scan_slot(tid * kScanV + i)] = run;
            run += v[i];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kScanV; ++j) {
            const int e = j * kBlock + tid;
            if (e < m)
                row[base + e] = buf[scan_slot(e)];
        }
        carry += tot;
        __syncthreads();  // buf is refilled by the next round
    }
    if (tid == 0)
        totals[p] = carry;
}

// Block b: destination b mod D of table b / D.
__global__ __launch_bounds__(kBlock) void part_scan_tiles(int64_t *cnt0, int64_t ntiles0,
                                                          int64_t *totals0, int64_t *cnt1,
                                                          int64_t ntiles1, int64_t *totals1, int D)
{
    const bool second = (int)blockIdx.x >= D;
    scan_tiles_of(second ? cnt1 : cnt0, second ? ntiles1 : ntiles0, second ? totals1 : totals0,
                  second ? (int)blockIdx.x - D : (int)blockIdx.x);
}

// One table's destination offsets from its totals.
__device__ __forceinline__ void offsets_of(const int64_t *totals, int64_t *off, int P)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    int64_t carry = 0;
    for (int base = 0; base < P; base += kBlock) {
        const int p = base + threadIdx.x;
        const int64_t v = p < P ? totals[p] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(v, scratch, &tot);
        if (p < P)
            off[p] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0)
        off[P] = carry;
}

// Block t: table t's destination offsets.
__global__ __launch_bounds__(kBlock) void part_offsets(const int64_t *totals0, int64_t *off0,
                                                       const int64_t *totals1, int64_t *off1, int P)
{
    offsets_of(blockIdx.x ? totals1 : totals0, blockIdx.x ? off1 : off0, P);
}

// LDS carve-up of part_scatter (bytes, 16-byte aligned pieces).
struct ScatterLds {
    size_t stage_v, stage_k, stage_p, stage_d, whist, tstart, gbase, scratch, total;
};

__host__ __device__ inline size_t al16(size_t x)
{
    return (x + 15) & ~(size_t)15;
}

// dig: the tile also stages every row's next-pass digit byte.
__host__ __device__ inline ScatterLds scatter_lds(int T, int P, int key_bytes, bool dig)
{
    ScatterLds L;
    size_t o = 0;
    L.stage_v = o;
    o = al16(o + (size_t)T * 8);
    L.stage_k = o;
    o = al16(o + (size_t)T * key_bytes);
    L.stage_p = o;
    o = al16(o + (size_t)T * 2);
    L.stage_d = o;  // next-pass digit bytes (when they are written)
    o = al16(o + (dig ? (size_t)T : 0));
    L.whist = o;  // 16-bit counts: a tile holds at most 4096 rows
    o = al16(o + (size_t)kWavesPerBlock * P * 2);
    L.tstart = o;
    o = al16(o + (size_t)P * 4);
    L.gbase = o;
    o = al16(o + (size_t)P * 8);
    L.scratch = o;
    o = al16(o + (size_t)kWavesPerBlock * 8);
    L.total = o;
    return L;
}

// Exclusive prefix over a[0..P) in LDS, in place (all threads call).
__device__ inline void lds_excl_scan_u32(uint32_t *a, int P, int64_t *scratch)
{
    int64_t carry = 0;
    for (int base = 0; base < P; base += kBlock) {
        const int p = base + threadIdx.x;
        const int64_t v = p < P ? a[p] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(v, scratch, &tot);
        if (p < P)
            a[p] = (uint32_t)(carry + ex);
        carry += tot;
    }
    __syncthreads();
}

// Stable scatter of one tile, rows [row0, row_end) (at most kBlock R of them).
// A row's destination in [0, D) is dfn(fmix64(key)); with DIG_OUT every
// output row's next-pass digit digit_of(h, dshift, dbits) is written beside
// it (from the same hash).  base_of(d) is the output position of the tile's
// first row with destination d.  Wave w owns the contiguous rows
// [row0 + 64 R w, row0 + 64 R (w+1)); step c reads 64 consecutive rows.
// (The second pass hashes its keys again rather than reading the digit
// bytes: byte loads, 64 bytes per wave instruction, slowed it by a quarter.)
template <typename K, int R, bool DIG_OUT, typename DestFn, typename BaseFn>
__device__ __forceinline__ void scatter_tile(const K *__restrict__ keys,
                                             const int64_t *__restrict__ pay, int64_t row0,
                                             int64_t row_end, int D, int nbits, DestFn dfn,
                                             BaseFn base_of, K *__restrict__ keys_out,
                                             int64_t *__restrict__ pay_out, unsigned char *smem,
                                             uint8_t *__restrict__ dig_out, int dshift, int dbits)
{
    constexpr int T = kBlock * R;
    static_assert(T <= 65535, "per-wave tile counts are 16-bit");
    const ScatterLds L = scatter_lds(T, D, (int)sizeof(K), DIG_OUT);
    int64_t *stage_v = (int64_t *)(smem + L.stage_v);
    K *stage_k = (K *)(smem + L.stage_k);
    uint16_t *stage_p = (uint16_t *)(smem + L.stage_p);
    uint8_t *stage_d = (uint8_t *)(smem + L.stage_d);
    uint16_t *whist = (uint16_t *)(smem + L.whist);
    uint32_t *tstart = (uint32_t *)(smem + L.tstart);
    int64_t *gbase = (int64_t *)(smem + L.gbase);
    int64_t *scratch = (int64_t *)(smem + L.scratch);

    const int tid = threadIdx.x, w = tid / kWave, lane = tid & (kWave - 1);

    // The row loads go first (keys, then payloads, which are needed only
    // for staging), so that the destination bases' loads and the ranking
    // overlap them.
    const int64_t wrow0 = row0 + (int64_t)w * kWave * R;
    K kr[R];
    int64_t vr[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int64_t r = wrow0 + (int64_t)c * kWave + lane;
        kr[c] = r < row_end ? __builtin_nontemporal_load(keys + r) : K(0);
    }
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int64_t r = wrow0 + (int64_t)c * kWave + lane;
        vr[c] = r < row_end ? __builtin_nontemporal_load(pay + r) : 0;
    }
    for (int i = tid; i < kWavesPerBlock * D; i += kBlock)
        whist[i] = 0;
    for (int p = tid; p < D; p += kBlock)
        gbase[p] = base_of(p);
    __syncthreads();

    // Rank every row among the earlier rows of its wave with its destination.
    uint16_t *wh = whist + w * D;
    uint32_t pr[R], rk[R];
    uint8_t dg[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int64_t r = wrow0 + (int64_t)c * kWave + lane;
        const bool valid = r < row_end;
        const uint64_t h = fmix64(key_bits(kr[c]));
        const uint32_t p = valid ? dfn(h) : 0u;
        if (DIG_OUT)
            dg[c] = (uint8_t)digit_of(h, dshift, dbits);
        uint64_t m = ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (p >> b) & 1u;
            const uint64_t bb = ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = mbcnt(m);
        uint32_t prev = 0;
        if (valid)
            prev = wh[p];
        if (valid && rank == 0)
            wh[p] = (uint16_t)(prev + (uint32_t)__popcll(m));
        pr[c] = valid ? p : 0xffffffffu;
        rk[c] = prev + rank;
    }
    __syncthreads();

    // Per destination: tile count, and every wave's offset inside it.
    for (int p = tid; p < D; p += kBlock) {
        uint32_t acc = 0;
#pragma unroll
        for (int ww = 0; ww < kWavesPerBlock; ++ww) {
            const uint32_t c = whist[ww * D + p];
            whist[ww * D + p] = (uint16_t)acc;
            acc += c;
        }
        tstart[p] = acc;
    }
    __syncthreads();
    lds_excl_scan_u32(tstart, D, scratch);  // tstart[p]: first staged row of p
    for (int p = tid; p < D; p += kBlock) {
        const uint32_t t0 = tstart[p];
#pragma unroll
        for (int ww = 0; ww < kWavesPerBlock; ++ww)
            whist[ww * D + p] = (uint16_t)(whist[ww * D + p] + t0);
    }
    __syncthreads();

#pragma unroll
    for (int c = 0; c < R; ++c) {
        if (pr[c] != 0xffffffffu) {
            const uint32_t s = wh[pr[c]] + rk[c];
            stage_k[s] = kr[c];
            stage_v[s] = vr[c];
            stage_p[s] = (uint16_t)pr[c];
            if (DIG_OUT)
                stage_d[s] = dg[c];
        }
    }
    __syncthreads();

    const int rows = (int)((row_end - row0) < (int64_t)T ? (row_end - row0) : (int64_t)T);
    for (int s = tid; s < rows; s += kBlock) {
        const uint32_t p = stage_p[s];
        const int64_t dst = gbase[p] + (s - (int)tstart[p]);
        // Ordinary stores: a run's first and last cache lines are shared
        // with the neighbouring tiles' runs and must meet them in L2 (the
        // XCD-contiguous tile order keeps those tiles on one L2).  With
        // streaming stores the partial lines went to HBM separately: 25% more
        // bytes written, 26% slower at a fan-out of 128.
        keys_out[dst] = stage_k[s];
        pay_out[dst] = stage_v[s];
        if (DIG_OUT)
            dig_out[dst] = stage_d[s];
    }
}

// First-pass scatter of tile `tile` of table tb.
template <typename K, int R, bool DIG>
__device__ __forceinline__ void part_scatter_tile(const PartTable<K> &tb, int64_t tile,
                                                  const Dest &d, int dshift, int dbits,
                                                  unsigned char *smem)
{
    scatter_tile<K, R, DIG>(
        tb.keys, tb.pay, tile * (int64_t)(kBlock * R), tb.n, d.ndest, d.nbits,
        [&](uint64_t h) { return dest_of(h, d); },
        [&](int p) { return tb.off[p] + tb.cnt[(int64_t)p * tb.ntiles + tile]; }, tb.keys_out,
        tb.pay_out, smem, tb.dig, dshift, dbits);
}

template <typename K, int R, bool DIG>
__global__ __launch_bounds__(kBlock) void part_scatter(PartPair<K> T, Dest d, int dshift, int dbits)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t g = tile_of_block(blockIdx.x, gridDim.x);
    const bool second = g >= T.t[0].ntiles;
    part_scatter_tile<K, R, DIG>(pick(T, second), second ? g - T.t[0].ntiles : g, d, dshift,
                                 dbits, smem);
}

// ---- segmented partition -------------------------------------------------------
// Tiles of 4096 rows never straddle a segment; chunks of 8 tiles never
// straddle a segment.  A row's position is
//   outoff[a D + q] + (rows of (a, q) in earlier chunks of a)
//                   + (rows of (a, q) in earlier tiles of the chunk)
//                   + (rank inside the tile),
// i.e. the stable counting-sort position inside segment a.
template <typename K>
struct SegTable {
    const K *keys;
    const int64_t *pay;
    const uint8_t *dig;      // digit byte per row
    const int64_t *segoff;   // [nseg + 1]
    int64_t *tile_start;     // [nseg + 1]
    int64_t *chunk_start;    // [nseg + 1]
    uint32_t *cnt;           // [max_tiles][D]
    int64_t *csum;           // [max_chunks][D]
    int64_t *outoff;         // [nseg D + 1]
    uint32_t *tile_seg;      // [max_tiles]: segment of every tile
    uint32_t *chunk_seg;     // [max_chunks]: segment of every chunk
    K *keys_out;
    int64_t *pay_out;
    int64_t max_tiles, max_chunks;
};

template <typename K>
struct SegPair {
    SegTable<K> t[2];
};

template <typename K>
__device__ __forceinline__ SegTable<K> pick(const SegPair<K> &T, bool second)
{
    const SegTable<K> &a = T.t[0], &b = T.t[1];
    SegTable<K> r;
    r.keys = second ? b.keys : a.keys;
    r.pay = second ? b.pay : a.pay;
    r.dig = second ? b.dig : a.dig;
    r.segoff = second ? b.segoff : a.segoff;
    r.tile_start = second ? b.tile_start : a.tile_start;
    r.chunk_start = second ? b.chunk_start : a.chunk_start;
    r.cnt = second ? b.cnt : a.cnt;
    r.csum = second ? b.csum : a.csum;
    r.outoff = second ? b.outoff : a.outoff;
    r.tile_seg = second ? b.tile_seg : a.tile_seg;
    r.chunk_seg = second ? b.chunk_seg : a.chunk_seg;
    r.keys_out = second ? b.keys_out : a.keys_out;
    r.pay_out = second ? b.pay_out : a.pay_out;
    r.max_tiles = second ? b.max_tiles : a.max_tiles;
    r.max_chunks = second ? b.max_chunks : a.max_chunks;
    return r;
}

// Block t: tile and chunk starts of every segment of table t, and the
// segment of every chunk (a chunk then finds its segment with one load
// instead of a search over the starts; seg_scan writes the same for tiles).
template <typename K>
__device__ __forceinline__ void seg_plan_of(const SegTable<K> &tb, int nseg)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    int64_t tcarry = 0, ccarry = 0;
    for (int base = 0; base < nseg; base += kBlock) {
        const int a = base + threadIdx.x;
        int64_t nt = 0;
        if (a < nseg)
            nt = (tb.segoff[a + 1] - tb.segoff[a] + kSegTile - 1) / kSegTile;
        const int64_t nc = (nt + kSegChunkTiles - 1) / kSegChunkTiles;
        int64_t tt, ct;
        const int64_t te = block_excl_scan(nt, scratch, &tt);
        const int64_t ce = block_excl_scan(nc, scratch, &ct);
        if (a < nseg) {
            tb.tile_start[a] = tcarry + te;
            tb.chunk_start[a] = ccarry + ce;
            for (int64_t c = 0; c < nc; ++c)
                tb.chunk_seg[ccarry + ce + c] = (uint32_t)a;
        }
        tcarry += tt;
        ccarry += ct;
    }
    if (threadIdx.x == 0) {
        tb.tile_start[nseg] = tcarry;
        tb.chunk_start[nseg] = ccarry;
    }
}

template <typename K>
__global__ __launch_bounds__(kBlock) void seg_plan(SegPair<K> T, int nseg)
{
    seg_plan_of(pick(T, blockIdx.x != 0), nseg);
}

// Block = chunk (the first table's max_chunks blocks, then the second's):
// per-tile digit counts, stored as the exclusive prefix over the chunk's
// earlier tiles; chunk totals to csum.  The digits are the bytes the first
// pass wrote beside its output rows, so this pass reads one byte per row
// instead of the key.  All of the chunk's bytes are loaded at once, four
// per load, then counted into one LDS histogram per tile.
template <typename K>
__device__ __forceinline__ void seg_hist_chunk(const SegTable<K> &tb, int64_t c, int nseg, int bits)
{
    __shared__ uint32_t hist[kSegChunkTiles][kSegMaxDest];
    static_assert(kSegTile == 4096, "tile of a row: (r - r0) >> 12");
    const int64_t nchunks = tb.chunk_start[nseg];
    const int a = (int)tb.chunk_seg[c];  // meaningful when c < nchunks
    if (c >= nchunks)
        return;
    const int D = 1 << bits, tid = threadIdx.x;
    const int64_t s1 = tb.segoff[a + 1];
    const int64_t t0 = tb.tile_start[a] + (c - tb.chunk_start[a]) * kSegChunkTiles;
    const int nt = (int)(t0 + kSegChunkTiles < tb.tile_start[a + 1] ? kSegChunkTiles
                                                                    : tb.tile_start[a + 1] - t0);
    const int64_t r0 = tb.segoff[a] + (t0 - tb.tile_start[a]) * kSegTile;  // chunk's first row
    const int64_t r1 = r0 + kSegChunkTiles * kSegTile < s1 ? r0 + kSegChunkTiles * kSegTile : s1;
    for (int i = tid; i < kSegChunkTiles * kSegMaxDest; i += kBlock)
        (&hist[0][0])[i] = 0;
    // The chunk's bytes as aligned 4-byte words: thread tid takes words
    // w0 + tid + j kBlock; a byte at row r counts toward tile (r - r0) / 4096
    // when r0 <= r < r1 (the digit array has 4 bytes of slack past its end).
    constexpr int kWords = (kSegChunkTiles * kSegTile / 4) / kBlock + 1;  // 17
    const int64_t w0 = r0 >> 2, w1 = (r1 + 3) >> 2;
    const uint32_t *words = (const uint32_t *)tb.dig;
    uint32_t dw[kWords];
#pragma unroll
    for (int j = 0; j < kWords; ++j) {
        const int64_t wi = w0 + tid + (int64_t)j * kBlock;
        dw[j] = wi < w1 ? __builtin_nontemporal_load(words + wi) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kWords; ++j) {
        const int64_t wi = w0 + tid + (int64_t)j * kBlock;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t r = 4 * wi + b;
            if (r >= r0 && r < r1)
                atomicAdd(&hist[(r - r0) >> 12][(dw[j] >> (8 * b)) & 0xffu], 1u);
        }
    }
    __syncthreads();
    for (int q = tid; q < D; q += kBlock) {
        uint32_t run = 0;
        for (int t = 0; t < nt; ++t) {
            tb.cnt[(t0 + t) * D + q] = run;
            run += hist[t][q];
        }
        tb.csum[c * D + q] = run;
    }
}

template <typename K>
__global__ __launch_bounds__(kBlock) void seg_hist(SegPair<K> T, int nseg, int bits)
{
    const bool second = (int64_t)blockIdx.x >= T.t[0].max_chunks;
    seg_hist_chunk(pick(T, second),
                   second ? (int64_t)blockIdx.x - T.t[0].max_chunks : (int64_t)blockIdx.x, nseg,
                   bits);
}

// Block = segment (nseg blocks per table): chunk totals -> exclusive prefix
// over the segment's chunks (in place); destination bases outoff[a D + q];
// the segment of each of the segment's tiles.
template <typename K>
__device__ __forceinline__ void seg_scan_of(const SegTable<K> &tb, int a, int nseg, int bits)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    __shared__ int64_t tot[kSegMaxDest];
    const int D = 1 << bits, tid = threadIdx.x;
    for (int64_t t = tb.tile_start[a] + tid; t < tb.tile_start[a + 1]; t += kBlock)
        tb.tile_seg[t] = (uint32_t)a;
    const int64_t c0 = tb.chunk_start[a], c1 = tb.chunk_start[a + 1];
    for (int q = tid; q < D; q += kBlock) {
        int64_t run = 0;
        for (int64_t c = c0; c < c1; ++c) {
            const int64_t v = tb.csum[c * D + q];
            tb.csum[c * D + q] = run;
            run += v;
        }
        tot[q] = run;
    }
    __syncthreads();
    int64_t carry = tb.segoff[a];
    for (int base = 0; base < D; base += kBlock) {
        const int q = base + tid;
        const int64_t v = q < D ? tot[q] : 0;
        int64_t all;
        const int64_t ex = block_excl_scan(v, scratch, &all);
        if (q < D)
            tb.outoff[(int64_t)a * D + q] = carry + ex;
        carry += all;
    }
    if (a == nseg - 1 && tid == 0)
        tb.outoff[(int64_t)nseg * D] = tb.segoff[nseg];
}

template <typename K>
__global__ __launch_bounds__(kBlock) void seg_scan(SegPair<K> T, int nseg, int bits)
{
    const bool second = (int)blockIdx.x >= nseg;
    seg_scan_of(pick(T, second), second ? (int)blockIdx.x - nseg : (int)blockIdx.x, nseg, bits);
}

// Block = tile (the first table's max_tiles, then the second's, in
// XCD-contiguous order over both).
template <typename K>
__device__ __forceinline__ void seg_scatter_tile(const SegTable<K> &tb, int64_t t, int nseg,
                                                 int shift, int bits, unsigned char *smem)
{
    const int64_t ntiles = tb.tile_start[nseg];
    const int a = (int)tb.tile_seg[t];  // meaningful when t < ntiles
    if (t >= ntiles)
        return;
    const int D = 1 << bits;
    const int64_t lt = t - tb.tile_start[a];
    const int64_t chunk = tb.chunk_start[a] + lt / kSegChunkTiles;
    const int64_t r0 = tb.segoff[a] + lt * kSegTile;
    const int64_t r1 = r0 + kSegTile < tb.segoff[a + 1] ? r0 + kSegTile : tb.segoff[a + 1];
    scatter_tile<K, kSegRows, false>(
        tb.keys, tb.pay, r0, r1, D, bits,
        [&](uint64_t h) { return digit_of(h, shift, bits); },
        [&](int q) {
            return tb.outoff[(int64_t)a * D + q] + tb.csum[chunk * D + q] +
                   (int64_t)tb.cnt[t * D + q];
        },
        tb.keys_out, tb.pay_out, smem, nullptr, 0, 0);
}

template <typename K>
__global__ __launch_bounds__(kBlock) void seg_scatter(SegPair<K> T, int nseg, int shift, int bits)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t g = tile_of_block(blockIdx.x, gridDim.x);
    const bool second = g >= T.t[0].max_tiles;
    seg_scatter_tile(pick(T, second), second ? g - T.t[0].max_tiles : g, nseg, shift, bits, smem);
}

// Kernel view of 1 or 2 tables partitioned into D destinations.
template <typename K>
PartPair<K> part_pair(const PartArgs *tables, int ntables, int D, int R)
{
    PartPair<K> T = {};
    for (int i = 0; i < ntables; ++i) {
        const PartArgs &a = tables[i];
        const PartLayout L = part_layout(a.n, D, R);
        PartTable<K> &t = T.t[i];
        t.keys = (const K *)a.keys;
        t.pay = a.pay;
        t.n = a.n;
        t.ntiles = L.ntiles;
        t.keys_out = (K *)a.keys_out;
        t.pay_out = a.pay_out;
        t.off = a.off;
        t.dig = a.dig;
        t.cnt = (int64_t *)((char *)a.ws + L.cnt_off);
        t.totals = (int64_t *)((char *)a.ws + L.totals_off);
    }
    return T;
}

template <typename K, int R>
hipError_t run_partition(const PartArgs *tables, int ntables, int32_t P, int sbits, int dshift,
                         int dbits, hipStream_t s)
{
    const Dest d = make_dest(P, sbits);
    const int D = d.ndest;
    const PartPair<K> T = part_pair<K>(tables, ntables, D, R);
    const int64_t tiles = T.t[0].ntiles + T.t[1].ntiles;
    if (tiles > 0) {
        trace_begin("part_hist", s);
        if (D <= kFewDest)
            hipLaunchKernelGGL((part_hist<K, R, true>), dim3((unsigned)tiles), dim3(kBlock),
                               (size_t)D * sizeof(uint32_t), s, T, d);
        else
            hipLaunchKernelGGL((part_hist<K, R, false>), dim3((unsigned)tiles), dim3(kBlock),
                               (size_t)D * sizeof(uint32_t), s, T, d);
        trace_end("part_hist", s);
    }
    hipLaunchKernelGGL(part_scan_tiles, dim3((unsigned)(D * ntables)), dim3(kBlock), 0, s,
                       T.t[0].cnt, T.t[0].ntiles, T.t[0].totals, T.t[1].cnt, T.t[1].ntiles,
                       T.t[1].totals, D);
    hipLaunchKernelGGL(part_offsets, dim3((unsigned)ntables), dim3(kBlock), 0, s, T.t[0].totals,
                       T.t[0].off, T.t[1].totals, T.t[1].off, D);
    if (tiles > 0) {
        // digit bytes are written for both tables or for neither
        const bool dig = T.t[0].dig != nullptr;
        const size_t lds = scatter_lds(kBlock * R, D, (int)sizeof(K), dig).total;
        if (lds > kMaxLdsBytes)
            return hipErrorInvalidValue;  // cannot happen for D <= MDX_MAX_P
        const void *fn = dig ? (const void *)part_scatter<K, R, true>
                             : (const void *)part_scatter<K, R, false>;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        trace_begin("part_scatter", s);
        if (dig)
            hipLaunchKernelGGL((part_scatter<K, R, true>), dim3((unsigned)tiles), dim3(kBlock), lds,
                               s, T, d, dshift, dbits);
        else
            hipLaunchKernelGGL((part_scatter<K, R, false>), dim3((unsigned)tiles), dim3(kBlock),
                               lds, s, T, d, dshift, dbits);
        trace_end("part_scatter", s);
    }
    return hipGetLastError();
}

// Kernel view of 1 or 2 tables split into nseg segments of 2^bits.
template <typename K>
SegPair<K> seg_pair(const SegArgs *tables, int ntables, int64_t nseg, int bits)
{
    SegPair<K> T = {};
    for (int i = 0; i < ntables; ++i) {
        const SegArgs &a = tables[i];
        const SegLayout L = seg_layout(a.n, nseg, bits);
        char *b = (char *)a.ws;
        SegTable<K> &t = T.t[i];
        t.keys = (const K *)a.keys;
        t.pay = a.pay;
        t.dig = a.dig;
        t.segoff = a.segoff;
        t.tile_start = (int64_t *)(b + L.tile_start_off);
        t.chunk_start = (int64_t *)(b + L.chunk_start_off);
        t.cnt = (uint32_t *)(b + L.cnt_off);
        t.csum = (int64_t *)(b + L.csum_off);
        t.outoff = a.outoff;
        t.tile_seg = (uint32_t *)(b + L.tile_seg_off);
        t.chunk_seg = (uint32_t *)(b + L.chunk_seg_off);
        t.keys_out = (K *)a.keys_out;
        t.pay_out = a.pay_out;
        t.max_tiles = L.max_tiles;
        t.max_chunks = L.max_chunks;
    }
    return T;
}

template <typename K>
hipError_t run_seg_partition(const SegArgs *tables, int ntables, int64_t nseg, int shift,
                             int bits, hipStream_t s)
{
    const SegPair<K> T = seg_pair<K>(tables, ntables, nseg, bits);
    const int ns = (int)nseg;
    const size_t lds = scatter_lds(kSegTile, 1 << bits, (int)sizeof(K), false).total;
    if (lds > kMaxLdsBytes)
        return hipErrorInvalidValue;  // cannot happen for bits <= 8
    hipLaunchKernelGGL(seg_plan<K>, dim3((unsigned)ntables), dim3(kBlock), 0, s, T, ns);
    trace_begin("seg_hist", s);
    hipLaunchKernelGGL(seg_hist<K>, dim3((unsigned)(T.t[0].max_chunks + T.t[1].max_chunks)),
                       dim3(kBlock), 0, s, T, ns, bits);
    trace_end("seg_hist", s);
    hipLaunchKernelGGL(seg_scan<K>, dim3((unsigned)(ns * ntables)), dim3(kBlock), 0, s, T, ns,
                       bits);
    hipError_t e = hipFuncSetAttribute((const void *)seg_scatter<K>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    trace_begin("seg_scatter", s);
    hipLaunchKernelGGL(seg_scatter<K>, dim3((unsigned)(T.t[0].max_tiles + T.t[1].max_tiles)),
                       dim3(kBlock), lds, s, T, ns, shift, bits);
    trace_end("seg_scatter", s);
    return hipGetLastError();
}

// ---- batches: one launch per step for many merges -----------------------------
// A batch launch covers every merge of a batch: merge m owns the blocks
// [pre[m], pre[m+1]) of the step's grid and reads its tables from record m
// (device memory).  The bodies are the ones the single launches run.
template <typename K>
struct PartRec {
    PartPair<K> T;  // build table, probe table
    Dest d;
    int32_t dshift, dbits;
};

template <typename K>
struct SegRec {
    SegPair<K> T;
    int32_t nseg, shift, bits, pad;
};

template <typename K, int R>
__global__ __launch_bounds__(kBlock) void part_hist_batch(const PartRec<K> *__restrict__ B,
                                                          const uint32_t *__restrict__ pre, int M)
{
    extern __shared__ uint32_t hist[];
    const uint32_t g = (uint32_t)tile_of_block(blockIdx.x, gridDim.x);
    const int m = find_range(pre, M, g);
    const PartRec<K> &r = B[m];
    const int64_t b = (int64_t)(g - pre[m]);
    const int second = b >= r.T.t[0].ntiles;
    hist_tile<K, R, true>(r.T.t[second], second ? b - r.T.t[0].ntiles : b, r.d, hist);
}

// One wave per (table, destination) -- merge m owns kWavesPerBlock of them
// per block, 2 D in all: a batch's tables mostly have few tiles, and a whole
// block per destination row left most of it idle.  The wave scans its row
// 64 kScanLane counts at a time, each lane kScanLane consecutive ones.
template <typename K>
__global__ __launch_bounds__(kBlock) void part_scan_batch(const PartRec<K> *__restrict__ B,
                                                          const uint32_t *__restrict__ pre, int M)
{
    const int m = find_range(pre, M, blockIdx.x);
    const PartRec<K> &r = B[m];
    const int lane = threadIdx.x & (kWave - 1);
    const int b = (int)(blockIdx.x - pre[m]) * kWavesPerBlock + (int)(threadIdx.x / kWave);
    const int D = r.d.ndest;
    if (b >= 2 * D)
        return;
    const int second = b >= D;
    const PartTable<K> &t = r.T.t[second];
    const int p = second ? b - D : b;
    const int64_t ntiles = t.ntiles;
    int64_t *row = t.cnt + (int64_t)p * ntiles;
    constexpr int kScanLane = 8;
    int64_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += (int64_t)kWave * kScanLane) {
        const int64_t i0 = base + (int64_t)lane * kScanLane;
        int64_t v[kScanLane], sum = 0;
#pragma unroll
        for (int j = 0; j < kScanLane; ++j) {
            v[j] = i0 + j < ntiles ? row[i0 + j] : 0;
            sum += v[j];
        }
        const int64_t inc = wave_incl_scan(sum, lane);
        int64_t run = carry + inc - sum;
#pragma unroll
        for (int j = 0; j < kScanLane; ++j) {
            if (i0 + j < ntiles)
                row[i0 + j] = run;
            run += v[j];
        }
        carry += __shfl(inc, kWave - 1, kWave);
    }
    if (lane == 0)
        t.totals[p] = carry;
}

template <typename K>
__global__ __launch_bounds__(kBlock) void part_offsets_batch(const PartRec<K> *__restrict__ B,
                                                             const uint32_t *__restrict__ pre,
                                                             int M)
{
    const int m = find_range(pre, M, blockIdx.x);
    const PartRec<K> &r = B[m];
    const PartTable<K> &t = r.T.t[blockIdx.x - pre[m]];
    offsets_of(t.totals, t.off, r.d.ndest);
}

template <typename K, int R>
__global__ __launch_bounds__(kBlock) void part_scatter_batch(const PartRec<K> *__restrict__ B,
                                                             const uint32_t *__restrict__ pre,
                                                             int M)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t g = (uint32_t)tile_of_block(blockIdx.x, gridDim.x);
    const int m = find_range(pre, M, g);
    const PartRec<K> &r = B[m];
    const int64_t b = (int64_t)(g - pre[m]);
    const int second = b >= r.T.t[0].ntiles;
    const PartTable<K> &t = r.T.t[second];
    const int64_t tile = second ? b - r.T.t[0].ntiles : b;
    if (t.dig)
        part_scatter_tile<K, R, true>(t, tile, r.d, r.dshift, r.dbits, smem);
    else
        part_scatter_tile<K, R, false>(t, tile, r.d, r.dshift, r.dbits, smem);
}

template <typename K>
__global__ __launch_bounds__(kBlock) void seg_plan_batch(const SegRec<K> *__restrict__ B,
                                                         const uint32_t *__restrict__ pre, int M)
{
    const int m = find_range(pre, M, blockIdx.x);
    const SegRec<K> &r = B[m];
    seg_plan_of(r.T.t[blockIdx.x - pre[m]], r.nseg);
}

template <typename K>
__global__ __launch_bounds__(kBlock) void seg_hist_batch(const SegRec<K> *__restrict__ B,
                                                         const uint32_t *__restrict__ pre, int M)
{
    const int m = find_range(pre, M, blockIdx.x);
    const SegRec<K> &r = B[m];
    const int64_t b = (int64_t)(blockIdx.x - pre[m]);
    const int second = b >= r.T.t[0].max_chunks;
    seg_hist_chunk(r.T.t[second], second ? b - r.T.t[0].max_chunks : b, r.nseg, r.bits);
}

template <typename K>
__global__ __launch_bounds__(kBlock) void seg_scan_batch(const SegRec<K> *__restrict__ B,
                                                         const uint32_t *__restrict__ pre, int M)
{
    const int m = find_range(pre, M, blockIdx.x);
    const SegRec<K> &r = B[m];
    const int b = (int)(blockIdx.x - pre[m]);
    const int second = b >= r.nseg;
    seg_scan_of(r.T.t[second], second ? b - r.nseg : b, r.nseg, r.bits);
}

template <typename K>
__global__ __launch_bounds__(kBlock) void seg_scatter_batch(const SegRec<K> *__restrict__ B,
                                                            const uint32_t *__restrict__ pre,
                                                            int M)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t g = (uint32_t)tile_of_block(blockIdx.x, gridDim.x);
    const int m = find_range(pre, M, g);
    const SegRec<K> &r = B[m];
    const int64_t b = (int64_t)(g - pre[m]);
    const int second = b >= r.T.t[0].max_tiles;
    seg_scatter_tile(r.T.t[second], second ? b - r.T.t[0].max_tiles : b, r.nseg, r.shift, r.bits,
                     smem);
}

template <typename K, int R>
hipError_t run_partition_batch(const void *recs, int M, int maxD, bool dig, BatchStage tiles,
                               BatchStage scan, BatchStage offs, hipStream_t s)
{
    const PartRec<K> *B = (const PartRec<K> *)recs;
    if (tiles.blocks > 0) {
        trace_begin("part_hist", s);
        hipLaunchKernelGGL((part_hist_batch<K, R>), dim3(tiles.blocks), dim3(kBlock),
                           (size_t)maxD * sizeof(uint32_t), s, B, tiles.pre, M);
        trace_end("part_hist", s);
    }
    if (scan.blocks > 0)
        hipLaunchKernelGGL(part_scan_batch<K>, dim3(scan.blocks), dim3(kBlock), 0, s, B, scan.pre,
                           M);
    if (offs.blocks > 0)
        hipLaunchKernelGGL(part_offsets_batch<K>, dim3(offs.blocks), dim3(kBlock), 0, s, B,
                           offs.pre, M);
    if (tiles.blocks > 0) {
        const size_t lds = scatter_lds(kBlock * R, maxD, (int)sizeof(K), dig).total;
        if (lds > kMaxLdsBytes)
            return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute((const void *)part_scatter_batch<K, R>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        trace_begin("part_scatter", s);
        hipLaunchKernelGGL((part_scatter_batch<K, R>), dim3(tiles.blocks), dim3(kBlock), lds, s, B,
                           tiles.pre, M);
        trace_end("part_scatter", s);
    }
    return hipGetLastError();
}

template <typename K>
hipError_t run_seg_batch(const void *recs, int M, int maxbits, BatchStage plan, BatchStage hist,
                         BatchStage scan, BatchStage tiles, hipStream_t s)
{
    const SegRec<K> *B = (const SegRec<K> *)recs;
    if (plan.blocks == 0)
        return hipSuccess;
    const size_t lds = scatter_lds(kSegTile, 1 << maxbits, (int)sizeof(K), false).total;
    if (lds > kMaxLdsBytes)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(seg_plan_batch<K>, dim3(plan.blocks), dim3(kBlock), 0, s, B, plan.pre, M);
    trace_begin("seg_hist", s);
    hipLaunchKernelGGL(seg_hist_batch<K>, dim3(hist.blocks), dim3(kBlock), 0, s, B, hist.pre, M);
    trace_end("seg_hist", s);
    hipLaunchKernelGGL(seg_scan_batch<K>, dim3(scan.blocks), dim3(kBlock), 0, s, B, scan.pre, M);
    hipError_t e = hipFuncSetAttribute((const void *)seg_scatter_batch<K>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    trace_begin("seg_scatter", s);
    hipLaunchKernelGGL(seg_scatter_batch<K>, dim3(tiles.blocks), dim3(kBlock), lds, s, B,
                       tiles.pre, M);
    trace_end("seg_scatter", s);
    return hipGetLastError();
}

template <typename K>
void write_part_rec(const PartArgs *tables, int32_t P, int sbits, int R, int dshift, int dbits,
                    void *dst)
{
    PartRec<K> r = {};
    r.d = make_dest(P, sbits);
    r.T = part_pair<K>(tables, 2, r.d.ndest, R);
    r.dshift = dshift;
    r.dbits = dbits;
    memcpy(dst, &r, sizeof(r));
}

template <typename K>
void write_seg_rec(const SegArgs *tables, int64_t nseg, int shift, int bits, void *dst)
{
    SegRec<K> r = {};
    r.T = seg_pair<K>(tables, 2, nseg, bits);
    r.nseg = (int32_t)nseg;
    r.shift = shift;
    r.bits = bits;
    memcpy(dst, &r, sizeof(r));
}

}  // namespace

hipError_t launch_partition(const PartArgs *tables, int ntables, int key_bytes, int32_t P,
                            int sbits, int dshift, int dbits, hipStream_t s)
{
    if (ntables < 1 || ntables > 2)
        return hipErrorInvalidValue;
    const bool small = part_rows_per_thread(P << sbits) == kPartRowsSmall;
    if (key_bytes == 8)
        return small ? run_partition<int64_t, kPartRowsSmall>(tables, ntables, P, sbits, dshift,
                                                              dbits, s)
                     : run_partition<int64_t, kPartRowsLarge>(tables, ntables, P, sbits, dshift,
                                                              dbits, s);
    return small ? run_partition<int32_t, kPartRowsSmall>(tables, ntables, P, sbits, dshift, dbits,
                                                          s)
                 : run_partition<int32_t, kPartRowsLarge>(tables, ntables, P, sbits, dshift, dbits,
                                                          s);
}

hipError_t launch_seg_partition(const SegArgs *tables, int ntables, int key_bytes, int64_t nseg,
                                int shift, int bits, hipStream_t s)
{
    if (ntables < 1 || ntables > 2)
        return hipErrorInvalidValue;
    if (key_bytes == 8)
        return run_seg_partition<int64_t>(tables, ntables, nseg, shift, bits, s);
    return run_seg_partition<int32_t>(tables, ntables, nseg, shift, bits, s);
}

}  // namespace mdx

namespace mdx {

size_t part_rec_bytes()
{
    static_assert(sizeof(PartRec<int32_t>) == sizeof(PartRec<int64_t>), "one record size");
    return sizeof(PartRec<int64_t>);
}

size_t seg_rec_bytes()
{
    static_assert(sizeof(SegRec<int32_t>) == sizeof(SegRec<int64_t>), "one record size");
    return sizeof(SegRec<int64_t>);
}

void part_rec(const PartArgs *tables, int key_bytes, int32_t P, int sbits, int R, int dshift,
              int dbits, void *dst)
{
    if (key_bytes == 8)
        write_part_rec<int64_t>(tables, P, sbits, R, dshift, dbits, dst);
    else
        write_part_rec<int32_t>(tables, P, sbits, R, dshift, dbits, dst);
}

void seg_rec(const SegArgs *tables, int key_bytes, int64_t nseg, int shift, int bits, void *dst)
{
    if (key_bytes == 8)
        write_seg_rec<int64_t>(tables, nseg, shift, bits, dst);
    else
        write_seg_rec<int32_t>(tables, nseg, shift, bits, dst);
}

hipError_t launch_partition_batch(const void *recs, int M, int key_bytes, int R, int maxD, bool dig,
                                  BatchStage tiles, BatchStage scan, BatchStage offs, hipStream_t s)
{
    if (R == kPartRowsSmall) {
        if (maxD > kPartSmallMaxP)
            return hipErrorInvalidValue;
        return key_bytes == 8
                   ? run_partition_batch<int64_t, kPartRowsSmall>(recs, M, maxD, dig, tiles, scan,
                                                                  offs, s)
                   : run_partition_batch<int32_t, kPartRowsSmall>(recs, M, maxD, dig, tiles, scan,
                                                                  offs, s);
    }
    if (R != kPartRowsLarge)
        return hipErrorInvalidValue;
    return key_bytes == 8
               ? run_partition_batch<int64_t, kPartRowsLarge>(recs, M, maxD, dig, tiles, scan, offs, s)
               : run_partition_batch<int32_t, kPartRowsLarge>(recs, M, maxD, dig, tiles, scan, offs,
                                                              s);
}

hipError_t launch_seg_batch(const void *recs, int M, int key_bytes, int maxbits, BatchStage plan,
                            BatchStage hist, BatchStage scan, BatchStage tiles, hipStream_t s)
{
    return key_bytes == 8
               ? run_seg_batch<int64_t>(recs, M, maxbits, plan, hist, scan, tiles, s)
               : run_seg_batch<int32_t>(recs, M, maxbits, plan, hist, scan, tiles, s);
}

}  // namespace mdx
