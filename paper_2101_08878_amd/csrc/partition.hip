// Stable hash partition of one table into P packed destination buffers.
//
// The shuffle's local half (arXiv 2101.08878, Section V-B, cuDF merge with
// "Shuffle: True"): each row goes to destination p = fmix64(key) mod P, and
// destination p's rows are packed, in input order, into [off[p], off[p+1]).
//
// Three passes over tiles of T = kBlock * R rows (512 x 8 = 4096):
//   part_hist       keys only: per-tile counts per destination (LDS atomics)
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
#include "mdx_internal.hpp"

namespace mdx {
namespace {

template <typename K, int R>
__global__ __launch_bounds__(kBlock) void part_hist(const K *__restrict__ keys, int64_t n, Dest d,
                                                    int64_t *__restrict__ cnt, int64_t ntiles)
{
    extern __shared__ uint32_t hist[];
    const int tid = threadIdx.x;
    const int P = d.ndest;  // destinations
    for (int p = tid; p < P; p += kBlock)
        hist[p] = 0;
    // XCD-contiguous tile order: the counts of neighbouring tiles share cache
    // lines, which then fill in one L2
    const int64_t tile = tile_of_block(blockIdx.x, gridDim.x);
    const int64_t row0 = tile * (int64_t)(kBlock * R);
    K k[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int64_t r = row0 + (int64_t)c * kBlock + tid;
        k[c] = r < n ? __builtin_nontemporal_load(keys + r) : K(0);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int64_t r = row0 + (int64_t)c * kBlock + tid;
        if (r < n)
            atomicAdd(&hist[dest_of(fmix64(key_bits(k[c])), d)], 1u);
    }
    __syncthreads();
    for (int p = tid; p < P; p += kBlock)
        cnt[(int64_t)p * ntiles + tile] = hist[p];
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

__global__ __launch_bounds__(kBlock) void part_scan_tiles(int64_t *__restrict__ cnt, int64_t ntiles,
                                                          int64_t *__restrict__ totals)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    __shared__ int64_t buf[kScanChunk + kBlock];
    const int tid = threadIdx.x;
    int64_t *row = cnt + (int64_t)blockIdx.x * ntiles;
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
        totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kBlock) void part_offsets(const int64_t *__restrict__ totals, int P,
                                                       int64_t *__restrict__ off)
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

// LDS carve-up of part_scatter (bytes, 16-byte aligned pieces).
struct ScatterLds {
    size_t stage_v, stage_k, stage_p, whist, tstart, gbase, scratch, total;
};

__host__ __device__ inline size_t al16(size_t x)
{
    return (x + 15) & ~(size_t)15;
}

__host__ __device__ inline ScatterLds scatter_lds(int T, int P, int key_bytes)
{
    ScatterLds L;
    size_t o = 0;
    L.stage_v = o;
    o = al16(o + (size_t)T * 8);
    L.stage_k = o;
    o = al16(o + (size_t)T * key_bytes);
    L.stage_p = o;
    o = al16(o + (size_t)T * 2);
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
// dfn(h) gives a row's destination in [0, D); base_of(d) the output position
// of the tile's first row with destination d.  Wave w owns the contiguous
// rows [row0 + 64 R w, row0 + 64 R (w+1)); step c reads 64 consecutive rows.
template <typename K, int R, typename DestFn, typename BaseFn>
__device__ __forceinline__ void scatter_tile(const K *__restrict__ keys,
                                             const int64_t *__restrict__ pay, int64_t row0,
                                             int64_t row_end, int D, int nbits, DestFn dfn,
                                             BaseFn base_of, K *__restrict__ keys_out,
                                             int64_t *__restrict__ pay_out, unsigned char *smem,
                                             uint8_t *__restrict__ dig_out = nullptr,
                                             int dshift = 0, int dbits = 0)
{
    constexpr int T = kBlock * R;
    static_assert(T <= 65535, "per-wave tile counts are 16-bit");
    const ScatterLds L = scatter_lds(T, D, (int)sizeof(K));
    int64_t *stage_v = (int64_t *)(smem + L.stage_v);
    K *stage_k = (K *)(smem + L.stage_k);
    uint16_t *stage_p = (uint16_t *)(smem + L.stage_p);
    uint16_t *whist = (uint16_t *)(smem + L.whist);
    uint32_t *tstart = (uint32_t *)(smem + L.tstart);
    int64_t *gbase = (int64_t *)(smem + L.gbase);
    int64_t *scratch = (int64_t *)(smem + L.scratch);

    const int tid = threadIdx.x, w = tid / kWave, lane = tid & (kWave - 1);
    for (int i = tid; i < kWavesPerBlock * D; i += kBlock)
        whist[i] = 0;
    for (int p = tid; p < D; p += kBlock)
        gbase[p] = base_of(p);

    const int64_t wrow0 = row0 + (int64_t)w * kWave * R;
    K kr[R];
    int64_t vr[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int64_t r = wrow0 + (int64_t)c * kWave + lane;
        const bool valid = r < row_end;
        kr[c] = valid ? __builtin_nontemporal_load(keys + r) : K(0);
        vr[c] = valid ? __builtin_nontemporal_load(pay + r) : 0;
    }
    __syncthreads();

    // Rank every row among the earlier rows of its wave with its destination.
    uint16_t *wh = whist + w * D;
    uint32_t pr[R], rk[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int64_t r = wrow0 + (int64_t)c * kWave + lane;
        const bool valid = r < row_end;
        const uint32_t p = valid ? dfn(fmix64(key_bits(kr[c]))) : 0u;
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
        if (dig_out)
            dig_out[dst] = (uint8_t)digit_of(fmix64(key_bits(stage_k[s])), dshift, dbits);
    }
}

template <typename K, int R>
__global__ __launch_bounds__(kBlock) void part_scatter(
    const K *__restrict__ keys, const int64_t *__restrict__ pay, int64_t n, Dest d,
    const int64_t *__restrict__ off, const int64_t *__restrict__ pre, int64_t ntiles,
    K *__restrict__ keys_out, int64_t *__restrict__ pay_out, uint8_t *__restrict__ dig_out,
    int dshift, int dbits)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t tile = tile_of_block(blockIdx.x, gridDim.x);
    scatter_tile<K, R>(
        keys, pay, tile * (int64_t)(kBlock * R), n, d.ndest, d.nbits,
        [&](uint64_t h) { return dest_of(h, d); },
        [&](int p) { return off[p] + pre[(int64_t)p * ntiles + tile]; }, keys_out, pay_out, smem,
        dig_out, dshift, dbits);
}

// ---- segmented partition -------------------------------------------------------
// Tiles of 4096 rows never straddle a segment; chunks of 8 tiles never
// straddle a segment.  A row's position is
//   outoff[a D + q] + (rows of (a, q) in earlier chunks of a)
//                   + (rows of (a, q) in earlier tiles of the chunk)
//                   + (rank inside the tile),
// i.e. the stable counting-sort position inside segment a.

__global__ __launch_bounds__(kBlock) void seg_plan(const int64_t *__restrict__ segoff, int nseg,
                                                   int64_t *__restrict__ tile_start,
                                                   int64_t *__restrict__ chunk_start)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    int64_t tcarry = 0, ccarry = 0;
    for (int base = 0; base < nseg; base += kBlock) {
        const int a = base + threadIdx.x;
        int64_t nt = 0;
        if (a < nseg)
            nt = (segoff[a + 1] - segoff[a] + kSegTile - 1) / kSegTile;
        const int64_t nc = (nt + kSegChunkTiles - 1) / kSegChunkTiles;
        int64_t tt, ct;
        const int64_t te = block_excl_scan(nt, scratch, &tt);
        const int64_t ce = block_excl_scan(nc, scratch, &ct);
        if (a < nseg) {
            tile_start[a] = tcarry + te;
            chunk_start[a] = ccarry + ce;
        }
        tcarry += tt;
        ccarry += ct;
    }
    if (threadIdx.x == 0) {
        tile_start[nseg] = tcarry;
        chunk_start[nseg] = ccarry;
    }
}

// Block = chunk: per-tile digit counts, stored as the exclusive prefix over
// the chunk's earlier tiles; chunk totals to csum.  The digits are the bytes
// the first pass wrote beside its output rows, so this pass reads one byte
// per row instead of the key.  All of the chunk's bytes are loaded at once,
// then counted into one LDS histogram per tile.
__global__ __launch_bounds__(kBlock) void seg_hist(
    const uint8_t *__restrict__ dig, const int64_t *__restrict__ segoff, int nseg,
    const int64_t *__restrict__ tile_start, const int64_t *__restrict__ chunk_start, int bits,
    uint32_t *__restrict__ cnt, int64_t *__restrict__ csum)
{
    __shared__ uint32_t hist[kSegChunkTiles][kSegMaxDest];
    constexpr uint32_t kNone = 0xffffffffu;
    const int64_t c = blockIdx.x;
    if (c >= chunk_start[nseg])
        return;
    const int D = 1 << bits, tid = threadIdx.x;
    const int a = upper_index(chunk_start, 0, nseg, c);
    const int64_t s1 = segoff[a + 1];
    const int64_t t0 = tile_start[a] + (c - chunk_start[a]) * kSegChunkTiles;
    const int nt = (int)(t0 + kSegChunkTiles < tile_start[a + 1] ? kSegChunkTiles
                                                                  : tile_start[a + 1] - t0);
    const int64_t r0 = segoff[a] + (t0 - tile_start[a]) * kSegTile;  // chunk's first row
    for (int i = tid; i < kSegChunkTiles * kSegMaxDest; i += kBlock)
        (&hist[0][0])[i] = 0;
    uint32_t d[kSegChunkTiles * kSegRows];
#pragma unroll
    for (int j = 0; j < kSegChunkTiles * kSegRows; ++j) {
        const int64_t r = r0 + (int64_t)j * kBlock + tid;  // tile j / kSegRows
        d[j] = r < s1 ? (uint32_t)__builtin_nontemporal_load(dig + r) : kNone;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSegChunkTiles * kSegRows; ++j)
        if (d[j] != kNone)
            atomicAdd(&hist[j / kSegRows][d[j]], 1u);
    __syncthreads();
    for (int q = tid; q < D; q += kBlock) {
        uint32_t run = 0;
        for (int t = 0; t < nt; ++t) {
            cnt[(t0 + t) * D + q] = run;
            run += hist[t][q];
        }
        csum[c * D + q] = run;
    }
}

// Block = segment: chunk totals -> exclusive prefix over the segment's chunks
// (in place); destination bases outoff[a D + q].
__global__ __launch_bounds__(kBlock) void seg_scan(const int64_t *__restrict__ segoff, int nseg,
                                                   const int64_t *__restrict__ chunk_start,
                                                   int bits, int64_t *__restrict__ csum,
                                                   int64_t *__restrict__ outoff)
{
    __shared__ int64_t scratch[kWavesPerBlock];
    __shared__ int64_t tot[kSegMaxDest];
    const int a = blockIdx.x, D = 1 << bits, tid = threadIdx.x;
    const int64_t c0 = chunk_start[a], c1 = chunk_start[a + 1];
    for (int q = tid; q < D; q += kBlock) {
        int64_t run = 0;
        for (int64_t c = c0; c < c1; ++c) {
            const int64_t v = csum[c * D + q];
            csum[c * D + q] = run;
            run += v;
        }
        tot[q] = run;
    }
    __syncthreads();
    int64_t carry = segoff[a];
    for (int base = 0; base < D; base += kBlock) {
        const int q = base + tid;
        const int64_t v = q < D ? tot[q] : 0;
        int64_t all;
        const int64_t ex = block_excl_scan(v, scratch, &all);
        if (q < D)
            outoff[(int64_t)a * D + q] = carry + ex;
        carry += all;
    }
    if (a == nseg - 1 && tid == 0)
        outoff[(int64_t)nseg * D] = segoff[nseg];
}

template <typename K>
__global__ __launch_bounds__(kBlock) void seg_scatter(
    const K *__restrict__ keys, const int64_t *__restrict__ pay,
    const int64_t *__restrict__ segoff, int nseg, const int64_t *__restrict__ tile_start,
    const int64_t *__restrict__ chunk_start, int shift, int bits,
    const uint32_t *__restrict__ cnt, const int64_t *__restrict__ csum,
    const int64_t *__restrict__ outoff, K *__restrict__ keys_out, int64_t *__restrict__ pay_out,
    const int32_t *gate)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (gate && *gate == 0)
        return;
    const int64_t t = tile_of_block(blockIdx.x, gridDim.x);
    if (t >= tile_start[nseg])
        return;
    const int D = 1 << bits;
    const int a = upper_index(tile_start, 0, nseg, t);
    const int64_t lt = t - tile_start[a];
    const int64_t chunk = chunk_start[a] + lt / kSegChunkTiles;
    const int64_t r0 = segoff[a] + lt * kSegTile;
    const int64_t r1 = r0 + kSegTile < segoff[a + 1] ? r0 + kSegTile : segoff[a + 1];
    scatter_tile<K, kSegRows>(
        keys, pay, r0, r1, D, bits,
        [&](uint64_t h) { return digit_of(h, shift, bits); },
        [&](int q) {
            return outoff[(int64_t)a * D + q] + csum[chunk * D + q] + (int64_t)cnt[t * D + q];
        },
        keys_out, pay_out, smem);
}

template <typename K, int R>
hipError_t run_partition(const K *keys, const int64_t *pay, int64_t n, int32_t P, int sbits,
                         K *keys_out, int64_t *pay_out, int64_t *off, uint8_t *dig_out,
                         int dshift, int dbits, void *ws, hipStream_t s)
{
    const Dest d = make_dest(P, sbits);
    const int D = d.ndest;
    const PartLayout L = part_layout(n, D);
    int64_t *cnt = (int64_t *)((char *)ws + L.cnt_off);
    int64_t *totals = (int64_t *)((char *)ws + L.totals_off);
    if (L.ntiles > 0) {
        trace_begin("part_hist", s);
        hipLaunchKernelGGL((part_hist<K, R>), dim3((unsigned)L.ntiles), dim3(kBlock),
                           (size_t)D * sizeof(uint32_t), s, keys, n, d, cnt, L.ntiles);
        trace_end("part_hist", s);
    }
    hipLaunchKernelGGL(part_scan_tiles, dim3((unsigned)D), dim3(kBlock), 0, s, cnt, L.ntiles,
                       totals);
    hipLaunchKernelGGL(part_offsets, dim3(1), dim3(kBlock), 0, s, totals, D, off);
    if (L.ntiles > 0) {
        const size_t lds = scatter_lds(kBlock * R, D, (int)sizeof(K)).total;
        if (lds > kMaxLdsBytes)
            return hipErrorInvalidValue;  // cannot happen for D <= MDX_MAX_P
        hipError_t e = hipFuncSetAttribute((const void *)part_scatter<K, R>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        trace_begin("part_scatter", s);
        hipLaunchKernelGGL((part_scatter<K, R>), dim3((unsigned)L.ntiles), dim3(kBlock), lds, s,
                           keys, pay, n, d, off, cnt, L.ntiles, keys_out, pay_out, dig_out,
                           dshift, dbits);
        trace_end("part_scatter", s);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_partition(const void *keys, const int64_t *pay, int64_t n, int key_bytes,
                            int32_t P, int sbits, void *keys_out, int64_t *pay_out, int64_t *off,
                            uint8_t *dig_out, int dshift, int dbits, void *ws, hipStream_t s)
{
    const int R = part_rows_per_thread(P << sbits);
    if (key_bytes == 8) {
        if (R == kPartRowsSmall)
            return run_partition<int64_t, kPartRowsSmall>((const int64_t *)keys, pay, n, P, sbits,
                                                          (int64_t *)keys_out, pay_out, off,
                                                          dig_out, dshift, dbits, ws, s);
        return run_partition<int64_t, kPartRowsLarge>((const int64_t *)keys, pay, n, P, sbits,
                                                      (int64_t *)keys_out, pay_out, off, dig_out,
                                                      dshift, dbits, ws, s);
    }
    if (R == kPartRowsSmall)
        return run_partition<int32_t, kPartRowsSmall>((const int32_t *)keys, pay, n, P, sbits,
                                                      (int32_t *)keys_out, pay_out, off, dig_out,
                                                      dshift, dbits, ws, s);
    return run_partition<int32_t, kPartRowsLarge>((const int32_t *)keys, pay, n, P, sbits,
                                                  (int32_t *)keys_out, pay_out, off, dig_out,
                                                  dshift, dbits, ws, s);
}

hipError_t launch_seg_partition(const void *keys, const int64_t *pay, const uint8_t *dig,
                                int64_t n, int key_bytes, const int64_t *segoff, int64_t nseg,
                                int shift, int bits, void *keys_out, int64_t *pay_out,
                                int64_t *outoff, void *ws, const int32_t *gate, hipStream_t s)
{
    const SegLayout L = seg_layout(n, nseg, bits);
    char *b = (char *)ws;
    int64_t *tile_start = (int64_t *)(b + L.tile_start_off);
    int64_t *chunk_start = (int64_t *)(b + L.chunk_start_off);
    uint32_t *cnt = (uint32_t *)(b + L.cnt_off);
    int64_t *csum = (int64_t *)(b + L.csum_off);
    const int ns = (int)nseg;
    hipLaunchKernelGGL(seg_plan, dim3(1), dim3(kBlock), 0, s, segoff, ns, tile_start, chunk_start);
    const size_t lds = scatter_lds(kSegTile, 1 << bits, key_bytes).total;
    if (lds > kMaxLdsBytes)
        return hipErrorInvalidValue;  // cannot happen for bits <= 8
    trace_begin("seg_hist", s);
    hipLaunchKernelGGL(seg_hist, dim3((unsigned)L.max_chunks), dim3(kBlock), 0, s, dig, segoff,
                       ns, tile_start, chunk_start, bits, cnt, csum);
    trace_end("seg_hist", s);
    hipLaunchKernelGGL(seg_scan, dim3((unsigned)ns), dim3(kBlock), 0, s, segoff, ns, chunk_start,
                       bits, csum, outoff);
    hipError_t e;
    trace_begin("seg_scatter", s);
    if (key_bytes == 8) {
        e = hipFuncSetAttribute((const void *)seg_scatter<int64_t>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(seg_scatter<int64_t>, dim3((unsigned)L.max_tiles), dim3(kBlock), lds, s,
                           (const int64_t *)keys, pay, segoff, ns, tile_start, chunk_start, shift,
                           bits, cnt, csum, outoff, (int64_t *)keys_out, pay_out, gate);
    } else {
        e = hipFuncSetAttribute((const void *)seg_scatter<int32_t>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(seg_scatter<int32_t>, dim3((unsigned)L.max_tiles), dim3(kBlock), lds, s,
                           (const int32_t *)keys, pay, segoff, ns, tile_start, chunk_start, shift,
                           bits, cnt, csum, outoff, (int32_t *)keys_out, pay_out, gate);
    }
    trace_end("seg_scatter", s);
    return hipGetLastError();
}

}  // namespace mdx
