// Internal host interface between the ABI layer (mdx_abi.cpp) and the kernel
// files (partition.hip, join.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mdx_device.hpp"

namespace mdx {

constexpr size_t kAlign = 256;
constexpr size_t kMaxLdsBytes = 160 * 1024;  // LDS of one gfx950 CU

inline size_t align_up(size_t x, size_t a = kAlign)
{
    return (x + a - 1) / a * a;
}

inline int ceil_log2(int64_t x)
{
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) < x)
        ++b;
    return b;
}

inline Dest make_dest(int32_t P, int sbits = 0)
{
    Dest d;
    d.P = (uint64_t)P;
    d.pow2 = (P & (P - 1)) == 0;
    d.mask = d.pow2 ? (uint64_t)(P - 1) : 0;
    d.sbits = sbits;
    d.ndest = P << sbits;
    d.nbits = ceil_log2(d.ndest);
    return d;
}

// ---- partition ------------------------------------------------------------
// Rows per tile of the partition kernels: kBlock threads x R rows.  Small P
// keeps one tile's rows staged in LDS; large P needs LDS for its counters.
#ifndef MDX_PART_ROWS
#define MDX_PART_ROWS 8
#endif
constexpr int kPartRowsSmall = MDX_PART_ROWS;  // tile kBlock R rows, P <= kPartSmallMaxP
constexpr int kPartRowsLarge = 2;    // tile 1024 rows (LDS holds 16-bit counts per wave and P)
constexpr int kPartSmallMaxP = 256;

inline int part_rows_per_thread(int32_t P)
{
    return P <= kPartSmallMaxP ? kPartRowsSmall : kPartRowsLarge;
}

struct PartLayout {
    int64_t ntiles;
    int rows_per_thread;
    size_t cnt_off, totals_off, bytes;
};

// R: rows per thread of the tiles (0: part_rows_per_thread(P)).
inline PartLayout part_layout(int64_t n, int32_t P, int R = 0)
{
    PartLayout L;
    L.rows_per_thread = R > 0 ? R : part_rows_per_thread(P);
    const int64_t tile = (int64_t)kBlock * L.rows_per_thread;
    L.ntiles = (n + tile - 1) / tile;
    size_t o = 0;
    L.cnt_off = o;
    o += align_up((size_t)P * (size_t)L.ntiles * sizeof(int64_t));
    L.totals_off = o;
    o += align_up((size_t)P * sizeof(int64_t));
    L.bytes = o;
    return L;
}

// One table of a partition launch: stable partition into
// make_dest(P, sbits).ndest destinations; off has ndest + 1 entries; ws holds
// part_layout(n, ndest).bytes.  With dig (n bytes), every output row's
// digit_of(h, dshift, dbits) is written beside it, for the histogram of a
// following segmented pass.
struct PartArgs {
    const void *keys;
    const int64_t *pay;
    int64_t n;
    void *keys_out;
    int64_t *pay_out;
    int64_t *off;
    uint8_t *dig;
    void *ws;
};

// Partition 1 or 2 tables (same key width and destinations) with one set of
// launches.
hipError_t launch_partition(const PartArgs *tables, int ntables, int key_bytes, int32_t P,
                            int sbits, int dshift, int dbits, hipStream_t s);

// ---- segmented partition (second split of the join) -------------------------
// Segment a (rows [segoff[a], segoff[a+1]) of an already partitioned table)
// is split stably into 2^bits destinations by digit_of(h, shift, bits);
// destination (a, q) lands at [outoff[a 2^bits + q], outoff[a 2^bits + q + 1]).
#ifndef MDX_SEG_ROWS
#define MDX_SEG_ROWS 8
#endif
constexpr int kSegRows = MDX_SEG_ROWS;          // rows per thread
constexpr int kSegTile = kBlock * kSegRows;     // 4096 rows per tile
constexpr int kSegChunkTiles = 8;               // tiles per scan chunk
constexpr int kSegMaxDest = 256;

struct SegLayout {
    int64_t max_tiles, max_chunks;
    size_t tile_start_off, chunk_start_off, cnt_off, csum_off, tile_seg_off, chunk_seg_off, bytes;
};

inline SegLayout seg_layout(int64_t n, int64_t nseg, int bits)
{
    SegLayout L;
    const int64_t D = (int64_t)1 << bits;
    L.max_tiles = (n + kSegTile - 1) / kSegTile + nseg;
    L.max_chunks = L.max_tiles / kSegChunkTiles + nseg + 1;
    size_t o = 0;
    L.tile_start_off = o;
    o += align_up((size_t)(nseg + 1) * sizeof(int64_t));
    L.chunk_start_off = o;
    o += align_up((size_t)(nseg + 1) * sizeof(int64_t));
    L.cnt_off = o;
    o += align_up((size_t)L.max_tiles * D * sizeof(uint32_t));
    L.csum_off = o;
    o += align_up((size_t)L.max_chunks * D * sizeof(int64_t));
    L.tile_seg_off = o;
    o += align_up((size_t)L.max_tiles * sizeof(uint32_t));
    L.chunk_seg_off = o;
    o += align_up((size_t)L.max_chunks * sizeof(uint32_t));
    L.bytes = o;
    return L;
}

// One table of a segmented launch: dig holds every row's
// digit_of(h, shift, bits), one byte per row (bits <= 8), 4-byte aligned and
// readable 4 bytes past its end (it is read as words); segoff has nseg + 1
// entries, outoff nseg 2^bits + 1; ws holds seg_layout(n, nseg, bits).bytes.
struct SegArgs {
    const void *keys;
    const int64_t *pay;
    const uint8_t *dig;
    int64_t n;
    const int64_t *segoff;
    void *keys_out;
    int64_t *pay_out;
    int64_t *outoff;
    void *ws;
};

// Split 1 or 2 tables (same key width, segment count and digits) with one
// set of launches.
hipError_t launch_seg_partition(const SegArgs *tables, int ntables, int key_bytes, int64_t nseg,
                                int shift, int bits, hipStream_t s);

// ---- batch launches -------------------------------------------------------------
// One launch of a step covers many merges: merge m owns blocks
// [pre[m], pre[m+1]) of the grid (pre in device memory, M + 1 entries,
// pre[M] = blocks) and reads its arguments from record m of a device array
// of records written on the host by the *_rec functions.
struct BatchStage {
    const uint32_t *pre;
    uint32_t blocks;
};

// Record of a merge's first pass over its two tables (tables[0] build,
// tables[1] probe) with tiles of kBlock R rows, as launch_partition would
// run it; part_rec_bytes() bytes.
size_t part_rec_bytes();
void part_rec(const PartArgs *tables, int key_bytes, int32_t P, int sbits, int R, int dshift,
              int dbits, void *dst);
// Record of a merge's segmented pass, as launch_seg_partition would run it.
size_t seg_rec_bytes();
void seg_rec(const SegArgs *tables, int key_bytes, int64_t nseg, int shift, int bits, void *dst);

// First pass of M merges of one key width and rows per thread R: `tiles`
// (both tables' tiles per merge), `scan` (ceil(2 D / kWavesPerBlock) per
// merge: a wave per table and destination), `offs` (2 per merge).  maxD: the largest destination count; dig: some merge writes
// digit bytes.
hipError_t launch_partition_batch(const void *recs, int M, int key_bytes, int R, int maxD, bool dig,
                                  BatchStage tiles, BatchStage scan, BatchStage offs, hipStream_t s);
// Segmented pass of the merges that have one (others own no blocks): `plan`
// (2 per merge), `hist` (max_chunks of both tables), `scan` (2 nseg),
// `tiles` (max_tiles of both tables); maxbits: the largest digit width.
hipError_t launch_seg_batch(const void *recs, int M, int key_bytes, int maxbits, BatchStage plan,
                            BatchStage hist, BatchStage scan, BatchStage tiles, hipStream_t s);

// ---- radix join (LDS tables per sub-bucket) ---------------------------------
// Sub-bucket s of S = P 2^qbits holds build rows [subL[s], subL[s+1]) and
// probe rows [subR[s], subR[s+1]); partition p owns sub-buckets
// [p 2^qbits, (p+1) 2^qbits).
// Two 512-thread workgroups per CU, each with a 77 KB table in LDS: the time
// of a sub-bucket is mostly the latency of its dependent steps (ticket,
// offsets, row loads, chained scan), and a second workgroup on the CU runs
// while the first waits.  (One workgroup with a 152 KB table for twice the
// rows, and so half the sub-buckets, was 10% slower at 1E8 x 1E8.)  A
// merge's table holds 3456 rows under 4096 chain heads: sub-buckets average
// 0.9 of it (so 1E8 rows in 32 partitions still make 32768 sub-buckets), and
// chains average under 0.8 rows (3840 rows under 2048 heads was 7% slower),
// so a thread walks the chains of two probe rows at a time (four: 2%
// slower).  The fused batch's join keeps 3840 rows under 2048 heads and
// walks four chains at a time: its mid-size merges (1E4 to 1E6 rows) gain
// more from 10% larger sub-buckets (fewer of them) than from shorter chains.
#ifndef MDX_JOIN_PER_CU
#define MDX_JOIN_PER_CU 2
#endif
#ifndef MDX_JOIN_CAP
#define MDX_JOIN_CAP 3456
#endif
#ifndef MDX_JOIN_HEADS
#define MDX_JOIN_HEADS 4096
#endif
#ifndef MDX_BATCH_JOIN_CAP
#define MDX_BATCH_JOIN_CAP 3840
#endif
#ifndef MDX_BATCH_JOIN_HEADS
#define MDX_BATCH_JOIN_HEADS 2048
#endif
#ifndef MDX_JOIN_ROWS
#define MDX_JOIN_ROWS 8
#endif
constexpr int kJoinPerCu = MDX_JOIN_PER_CU;
constexpr int kJoinThreads = 512;
// Geometry of a join workgroup's LDS table: build rows, chain heads, and
// the probe rows of a thread whose chains are walked together.
template <int CAP, int HEADS, int WALK>
struct JoinGeo {
    static constexpr int cap = CAP;
    static constexpr int heads = HEADS;
    static constexpr int walk = WALK;
};
using MergeJoin = JoinGeo<MDX_JOIN_CAP, MDX_JOIN_HEADS, 2>;             // rj_join
using BatchJoin = JoinGeo<MDX_BATCH_JOIN_CAP, MDX_BATCH_JOIN_HEADS, 4>;  // rj_join_batch
constexpr int kJoinCap = MergeJoin::cap;       // build rows per table of a merge
constexpr int kBatchJoinCap = BatchJoin::cap;  // ... of the fused batch
constexpr int kJoinRows = MDX_JOIN_ROWS;    // probe rows per thread per batch
constexpr int kJoinBatch = kJoinThreads * kJoinRows;
// Sub-buckets are sized for this fraction of a table on average (the larger
// side's rows): the largest of thousands stays below the cap (at ~3100 rows
// the cap is six standard deviations of a sub-bucket's size away).
#ifndef MDX_JOIN_FILL
#define MDX_JOIN_FILL 0.9
#endif
constexpr double kJoinFill = MDX_JOIN_FILL;

// One chained-scan tile per sub-bucket.
struct RJoinLayout {
    int64_t S;
    size_t status_off, tile_base_off, misc_off, bytes;
};

inline RJoinLayout rjoin_layout(int32_t P, int qbits)
{
    RJoinLayout L;
    L.S = (int64_t)P << qbits;
    size_t o = 0;
    L.status_off = o;
    o += align_up((size_t)L.S * sizeof(uint64_t));
    L.tile_base_off = o;
    o += align_up((size_t)L.S * sizeof(int64_t));
    L.misc_off = o;  // ticket (u32), use flag (i32)
    o += align_up(64);
    L.bytes = o;
    return L;
}

struct RJoinWs {
    uint64_t *status;
    int64_t *tile_base;
    uint32_t *ticket;
    int32_t *use;  // 1: every build sub-bucket fits an LDS table
    int64_t S;
};

inline RJoinWs rjoin_ws(void *base, const RJoinLayout &L)
{
    char *b = (char *)base;
    RJoinWs w;
    w.status = (uint64_t *)(b + L.status_off);
    w.tile_base = (int64_t *)(b + L.tile_base_off);
    w.ticket = (uint32_t *)(b + L.misc_off);
    w.use = (int32_t *)(b + L.misc_off + 16);
    w.S = L.S;
    return w;
}

// ---- join table -------------------------------------------------------------
// Partition p of a view over partitions [pb, pe) owns slots
//   [sb(p), sb(p) + 2 n_p + 16),  sb(p) = 2 (off[p] - off[pb]) + 16 (p - pb),
// split into two halves of H_p = n_p + 8 slots.  A key whose hash has top
// bit t lives in half t; half 0 marks empty slots with ~0 and half 1 with 0,
// values no hash of that half can take, so no key value is reserved.
struct TableLayout {
    size_t off_off, flags_off, bump_off, slots_off, gstart_off, grouped_off, bytes;
    int64_t nslots;
};

inline TableLayout table_layout(int64_t n, int32_t P)
{
    TableLayout L;
    L.nslots = 2 * n + 16 * (int64_t)P;
    size_t o = 0;
    L.off_off = o;
    o += align_up((size_t)(P + 1) * sizeof(int64_t));
    L.flags_off = o;
    o += align_up((size_t)P * sizeof(int32_t));
    L.bump_off = o;
    o += align_up((size_t)P * sizeof(int64_t));
    L.slots_off = o;
    o += align_up((size_t)L.nslots * 2 * sizeof(uint64_t));
    L.gstart_off = o;
    o += align_up((size_t)L.nslots * sizeof(int64_t));
    L.grouped_off = o;
    o += align_up((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    L.bytes = o;
    return L;
}

// Device view of the tables of partitions [pb, pe).
struct TView {
    uint64_t *slots;
    int64_t *gstart;
    int64_t *grouped;
    const int64_t *off;  // build offsets [P+1] (absolute rows)
    int32_t *flags;      // [P]
    int64_t *bump;       // [P]
    int32_t pb, pe;
    Dest d;
    const int32_t *skip;  // optional: kernels do nothing while *skip != 0
};

// ---- probe ------------------------------------------------------------------
constexpr int kProbeRows = 8;                       // rows per thread
constexpr int kProbeTile = kBlock * kProbeRows;     // 2048 rows per tile

struct Deferred {
    int64_t rbeg, rend;  // probe rows of the tile
    int64_t base, count; // output rows [base, base + count)
    int64_t group;
};

struct ProbeLayout {
    int64_t max_tiles;
    size_t off_off, tile_start_off, status_off, tile_base_off, ticket_off, ndefer_off, defer_off,
        row_pre_off, row_gs_off, bytes;
};

inline ProbeLayout probe_layout(int64_t n, int32_t P)
{
    ProbeLayout L;
    L.max_tiles = (n + kProbeTile - 1) / kProbeTile + P;
    size_t o = 0;
    L.off_off = o;
    o += align_up((size_t)(P + 1) * sizeof(int64_t));
    L.tile_start_off = o;
    o += align_up((size_t)(P + 1) * sizeof(int64_t));
    L.status_off = o;
    o += align_up((size_t)L.max_tiles * sizeof(uint64_t));
    L.tile_base_off = o;
    o += align_up((size_t)L.max_tiles * sizeof(int64_t));
    L.ticket_off = o;
    o += align_up((size_t)P * sizeof(uint32_t));
    L.ndefer_off = o;
    o += align_up(sizeof(uint32_t));
    L.defer_off = o;
    o += align_up((size_t)L.max_tiles * sizeof(Deferred));
    L.row_pre_off = o;
    o += align_up((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    L.row_gs_off = o;
    o += align_up((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    L.bytes = o;
    return L;
}

struct ProbeWs {
    int64_t *off;  // [P+1] sanitized probe offsets
    int64_t *tile_start;
    uint64_t *status;
    int64_t *tile_base;
    uint32_t *ticket;
    uint32_t *ndefer;
    Deferred *defer;
    int64_t *row_pre;
    int64_t *row_gs;
    int64_t max_tiles;
};

inline ProbeWs probe_ws(void *base, const ProbeLayout &L)
{
    char *b = (char *)base;
    ProbeWs w;
    w.off = (int64_t *)(b + L.off_off);
    w.tile_start = (int64_t *)(b + L.tile_start_off);
    w.status = (uint64_t *)(b + L.status_off);
    w.tile_base = (int64_t *)(b + L.tile_base_off);
    w.ticket = (uint32_t *)(b + L.ticket_off);
    w.ndefer = (uint32_t *)(b + L.ndefer_off);
    w.defer = (Deferred *)(b + L.defer_off);
    w.row_pre = (int64_t *)(b + L.row_pre_off);
    w.row_gs = (int64_t *)(b + L.row_gs_off);
    w.max_tiles = L.max_tiles;
    return w;
}

struct ProbeOut {
    void *key;
    int64_t *lpay;
    int64_t *rpay;
    int64_t cap;
    int64_t *offsets;  // [P+1]
};

// Number of workgroups that fill the device for grid-stride kernels.
int device_fill_blocks();

// Benchmark tracing (mdx_trace_kernel): the launch wrappers call these
// around the launches of the kernels that can be traced.
void trace_begin(const char *kernel, hipStream_t s);
void trace_end(const char *kernel, hipStream_t s);

// Build a view of `rows` rows: init slots, insert rows, group repeated keys.
// The grid-stride kernels of build and probe run on a full device, or on
// max_blocks workgroups when 0 < max_blocks < that.
hipError_t launch_build(const void *keys, const int64_t *pay, int key_bytes, const TView &v,
                        int64_t rows, int32_t *status, int max_blocks, hipStream_t s);

// Copy the build offsets (sanitized, for n build rows) into the table and
// clear per-partition flags.  off_in may be null (flags only).
hipError_t launch_table_setup(const int64_t *off_in, int64_t n, int64_t *off_tab, int32_t *flags,
                              int64_t *bump, int32_t P, hipStream_t s);

// A merge's global-table join set-up, in one launch (nothing when *skip):
// offPL / offPR[p] = offAL / offAR[p stride] (per-partition offsets from the
// first pass's), then launch_table_setup(offPL, n_build, ...) and
// launch_probe_plan(offPR, n_probe, ...).
hipError_t launch_fallback_setup(const int64_t *offAL, const int64_t *offAR, int stride,
                                 int32_t P, int64_t n_build, int64_t n_probe, int64_t *offPL,
                                 int64_t *offPR, int64_t *off_tab, int32_t *flags, int64_t *bump,
                                 const ProbeWs &w, const int32_t *skip, hipStream_t s);

// Probe: plan tiles from the probe offsets (sanitized for n probe rows, once
// per probe), probe one view (group g), finalize the output offsets.
hipError_t launch_probe_plan(const int64_t *offR, int64_t n, int32_t P, const ProbeWs &w,
                             const int32_t *skip, hipStream_t s);
hipError_t launch_probe_group(const void *pkeys, const int64_t *ppay, int key_bytes, int32_t P,
                              const TView &v, int group, const ProbeWs &w, const ProbeOut &o,
                              int32_t *status, int max_blocks, hipStream_t s);
hipError_t launch_probe_finalize(int32_t P, const ProbeWs &w, const ProbeOut &o,
                                 const int32_t *skip, hipStream_t s);

// Count-only join of two partitioned tables (full views, pb = 0, pe = P):
// per-partition output counts into out_offsets (exclusive prefix, total at
// [P]).  v: a table view (off, slots; v.off is written with the sanitized
// build offsets); off_probe [P+1] and pcount [P] are workspace.
hipError_t launch_join_count(const void *lk, const int64_t *lofs, int64_t n_build, const void *rk,
                             const int64_t *rofs, int64_t n_probe, int key_bytes, const TView &v,
                             int64_t *off_probe, uint64_t *pcount, int64_t *out_offsets,
                             int32_t *status, hipStream_t s);

// Radix join: plan (the LDS-fit flag from the build sub-buckets, cleared
// chained scan), join, output offsets.  chunked: a build sub-bucket larger
// than a table is joined in table-sized chunks (the flag stays set and no
// global-table join is needed); otherwise such a sub-bucket clears the flag
// and the join does nothing.
hipError_t launch_rjoin_plan(const int64_t *subL, const int64_t *subR, int64_t S,
                             const RJoinWs &w, bool chunked, hipStream_t s);
hipError_t launch_rjoin(const void *lk, const int64_t *lv, const int64_t *subL, const void *rk,
                        const int64_t *rv, const int64_t *subR, int key_bytes, int32_t P,
                        int qbits, const RJoinWs &w, const ProbeOut &o, int32_t *status,
                        bool chunked, hipStream_t s);
// Radix join of every merge of a batch (one key width): record m describes
// merge m (its S sub-buckets, its chained scan jstatus/jbase of S entries,
// output); Spre [M + 1] prefix of the merges' S in device memory, S its
// total; ticket: a device counter.  Clears the chained scans, joins (a build
// sub-bucket larger than an LDS table is joined in table-sized chunks), and
// writes every merge's output offsets.
struct JoinRec {
    const void *lk;
    const int64_t *lv;
    const int64_t *subL;  // [S + 1]
    const void *rk;
    const int64_t *rv;
    const int64_t *subR;  // [S + 1]
    uint64_t *jstatus;    // [S]
    int64_t *jbase;       // [S]
    int64_t S;
    ProbeOut o;
    int32_t *status;
    int32_t P, qbits;
    int32_t by_part;  // rjoin_by_partition: rows placed by partition cursor
    int32_t pad;
};

// Workgroups of a radix-join launch over S sub-buckets.
int rjoin_grid(int64_t S);

// Whether a radix join places its output rows by partition (a cursor per
// partition and a chained scan over partitions) rather than by sub-bucket
// (a chained scan over sub-buckets): when a partition's 2^qbits sub-buckets
// are many times the G workgroups working at once.
bool rjoin_by_partition(int qbits, int64_t G);

hipError_t launch_rjoin_batch(const JoinRec *recs, int M, const uint32_t *Spre, uint32_t S,
                              uint32_t *ticket, int key_bytes, hipStream_t s);

// A merge's output offsets: the radix join's when it ran, else (pw non-null)
// the global-table probe's.
hipError_t launch_merge_finalize(int32_t P, int qbits, const RJoinWs &w, const ProbeWs *pw,
                                 const ProbeOut &o, hipStream_t s);


// ---- transpose sum (y = x + x^T, float64) -------------------------------------------
hipError_t launch_transpose_sum(const double *x, double *y, int64_t n, hipStream_t s);

}  // namespace mdx
