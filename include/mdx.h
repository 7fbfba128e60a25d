/*
 * mdx.h -- C ABI of libmdx: the data-parallel work one Dask worker does in
 * the cuDF-merge benchmark of arXiv 2101.08878, on one MI355X (gfx950).
 *
 * The paper's workers shuffle both data frames on the join key and then
 * merge what they received (Section V-B "cuDF Merge"; the RI2 cuDF figure's
 * caption: chunk 1E8 rows, "Shuffle: True", fraction match 0.3; 3.2 GB per
 * worker, i.e. an int64 key and an int64 payload per row).  The shuffle's
 * local half is a hash partition of each table into P packed per-destination
 * buffers -- the device buffers the paper's MPI4Dask layer ships with
 * Isend/Irecv (Section IV-B, "Point-to-point Communication Coroutines", which
 * sends raw device buffers without serialization).  The merge is an inner
 * hash join of the partitions.  Inter-worker communication itself is not
 * part of this library.
 *
 * Conventions for every entry point:
 *  - Every function returns an int32 status (MDX_OK = 0).  No C++ exception
 *    crosses the ABI.  On a non-OK status, mdx_last_error() returns a
 *    thread-local message.
 *  - All device memory is owned by the caller.  libmdx never allocates or
 *    frees device memory; buffers whose size depends on the data are bounded
 *    by a *_bytes() query that depends only on sizes (n, P, key type).  The
 *    one exception is the fixed scratch array that the code object of
 *    mdx_hash_partition_noalloc carries (see there).
 *  - Device pointers ("d_" prefix) must point to memory of the current HIP
 *    device and be aligned to 256 bytes where they are workspaces or tables,
 *    and to their element size otherwise.  Host pointers have an "h_" prefix.
 *  - Work is enqueued asynchronously on the given hipStream_t (NULL = the
 *    null stream); no call synchronizes.  Arguments are validated on the host
 *    before anything is enqueued: a call that returns an error has enqueued
 *    nothing.
 *  - Keys are int32 (MDX_KEY_I32) or int64 (MDX_KEY_I64); payloads are int64.
 *    Keys are compared as exact integers over their full range (no sentinel
 *    value is reserved).  int32 keys are sign-extended to int64 before
 *    hashing, so an int32 and an int64 key of equal value share a partition.
 *  - The destination of a key is p = fmix64(key) mod P, where fmix64 is the
 *    64-bit finalizer of MurmurHash3 applied to the key's two's-complement
 *    bits and mod is the unsigned 64-bit remainder.  (The paper does not name
 *    its shuffle hash; this one is fixed here.)
 *  - Conditions only the device can see (an output larger than its
 *    capacity, a build table whose input is not partitioned as its offsets
 *    claim) are reported by OR-ing MDX_DEV_* bits into the caller's int32
 *    d_status word, which the caller zeroes before the first call and reads
 *    after synchronizing the stream.  d_status may be NULL.
 *  - Calls that share a workspace or a table must be ordered (same stream or
 *    explicit events); concurrent calls on different buffers are
 *    independent.
 */
#ifndef MDX_H
#define MDX_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MDX_ABI_VERSION 3

/* Largest number of partitions (destinations). */
#define MDX_MAX_P 4096
/* Largest number of rows in one table (2^34). */
#define MDX_MAX_ROWS (INT64_C(1) << 34)

/* Return statuses. */
#define MDX_OK 0
#define MDX_ERR_INVALID 1   /* a null pointer with n > 0, n < 0 or too large,
                               P outside [1, MDX_MAX_P], bad key type,
                               overlapping input/output, misaligned buffer */
#define MDX_ERR_WORKSPACE 2 /* workspace or table smaller than its *_bytes() */
#define MDX_ERR_HIP 3       /* a HIP runtime call or kernel launch failed */
#define MDX_BUSY 4          /* not an error: mdx_server_submit found no free
                               slot or memory budget; nothing was enqueued */

/* Key types: the value is the key width in bytes. */
#define MDX_KEY_I32 4
#define MDX_KEY_I64 8

/* Device-side status bits OR-ed into *d_status. */
#define MDX_DEV_OUTPUT_OVERFLOW 1 /* join output exceeded out_capacity; rows
                                     past the capacity were not written */
#define MDX_DEV_BAD_PARTITIONING 2 /* a row's destination did not match the
                                      partition its offsets place it in; the
                                      row was skipped */
#define MDX_DEV_SCAN_TIMEOUT 4     /* internal guard: the probe's chained
                                      scan waited too long for a predecessor
                                      tile; output offsets are unreliable.
                                      Never expected; reported instead of
                                      hanging the device. */

/* ABI version compiled into the library (MDX_ABI_VERSION). */
int32_t mdx_abi_version(void);

/* Static description of a status code; never NULL. */
const char *mdx_status_string(int32_t status);

/* Thread-local message about the last failing call on this thread ("" if
 * none).  Valid until the next libmdx call on the same thread. */
const char *mdx_last_error(void);

/* ---------------------------------------------------------------------------
 * Hash partition (the local half of the shuffle).
 *
 * Section V-B ("cuDF Merge", shuffle on): each worker splits its frame by a
 * hash of the join key into one packed buffer per destination worker, the
 * buffers Section IV-B's Isend/Irecv coroutines then ship as raw device
 * memory.
 * Stable partition of one table by p = fmix64(key) mod P.  On return (once
 * the stream reaches it):
 *   d_offsets[0] = 0, d_offsets[P] = n, and destination p's rows occupy
 *   [d_offsets[p], d_offsets[p+1]) of d_keys_out and d_payload_out, in
 *   their input order.  The result is unique, hence deterministic.
 * Arguments:
 *   d_keys [n] (key_type), d_payload [n] int64: input columns (read only).
 *   d_keys_out [n] (key_type), d_payload_out [n] int64: outputs; must not
 *     overlap the inputs.
 *   d_offsets [P+1] int64: output.
 *   d_ws: workspace of at least mdx_hash_partition_workspace_bytes(n, P,
 *     key_type) bytes; contents on entry are ignored.
 * n == 0 is valid (offsets all zero).  P > n is valid (empty destinations).
 * ------------------------------------------------------------------------- */
int32_t mdx_hash_partition_workspace_bytes(int64_t n, int32_t P, int32_t key_type,
                                           size_t *h_bytes);

int32_t mdx_hash_partition(const void *d_keys, const int64_t *d_payload, int64_t n,
                           int32_t key_type, int32_t P, void *d_keys_out,
                           int64_t *d_payload_out, int64_t *d_offsets, void *d_ws,
                           size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Hash partition without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).
 *
 * Computes exactly what mdx_hash_partition computes (same outputs, same
 * arguments minus the workspace).  Its workspace is a device array inside
 * the library of MDX_NOALLOC_SCRATCH_BYTES bytes: every GPU the library runs
 * on holds one, from the first call on that GPU until the process ends.  The
 * call itself allocates nothing (no hipMalloc, no allocating library call);
 * the caller still passes the input and output buffers.
 * Errors: as mdx_hash_partition, and MDX_ERR_WORKSPACE (nothing enqueued)
 * when mdx_hash_partition_workspace_bytes(n, P, key_type) exceeds
 * MDX_NOALLOC_SCRATCH_BYTES (e.g. n = 1E8 rows fits up to P = 85).
 * Every call on one GPU uses that GPU's one array: calls that overlap on a
 * GPU (different streams, or threads, without ordering between them) race
 * and give wrong results; order them.
 * ------------------------------------------------------------------------- */
#define MDX_NOALLOC_SCRATCH_BYTES (16u << 20)

int32_t mdx_hash_partition_noalloc(const void *d_keys, const int64_t *d_payload, int64_t n,
                                   int32_t key_type, int32_t P, void *d_keys_out,
                                   int64_t *d_payload_out, int64_t *d_offsets,
                                   hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Join build: one hash table per partition of the build (left) table.
 *
 * Section V-B ("cuDF Merge"): after the shuffle each worker merges the left
 * and right rows it received for its key range; this is the build half of
 * that inner hash join, over every destination partition at once.
 * The build input is a table partitioned by mdx_hash_partition (rows of
 * destination p in [d_offsets[p], d_offsets[p+1])).  The table memory
 * d_table_mem (caller-owned, at least mdx_join_table_bytes(n, P, key_type)
 * bytes) receives, per partition, an open-addressing table of the hashed keys
 * and, where a partition holds a repeated key, the build payloads grouped by
 * key.  The build copies d_offsets into the table, so the caller may reuse
 * d_keys, d_payload and d_offsets afterwards; d_table_mem must stay alive and
 * unchanged while the table is probed.
 * *h_table is a plain struct filled on the host (no device access); it
 * describes where things live inside d_table_mem.  There is nothing to
 * destroy: freeing d_table_mem ends the table.
 * A row whose destination differs from the partition its offsets place it in
 * is skipped (not inserted) and reported with MDX_DEV_BAD_PARTITIONING.
 * ------------------------------------------------------------------------- */
typedef struct mdx_table {
    int32_t abi_version; /* MDX_ABI_VERSION of the library that built it */
    int32_t P;
    int32_t key_type;
    int32_t reserved;
    int64_t n;           /* build rows */
    void *d_mem;         /* the caller's table memory */
    size_t bytes;        /* its size */
    /* Internal layout inside d_mem (read-only for the caller). */
    int64_t *d_offsets;  /* [P+1] copy of the build offsets */
    int32_t *d_flags;    /* [P] 1 if the partition has a repeated key */
    int64_t *d_bump;     /* [P] group allocator */
    uint64_t *d_slots;   /* [2 * (2n + 16P)] (hash, value) slot pairs */
    int64_t *d_gstart;   /* [2n + 16P] group start per slot */
    int64_t *d_grouped;  /* [n] payloads grouped by key */
} mdx_table;

int32_t mdx_join_table_bytes(int64_t n_build, int32_t P, int32_t key_type, size_t *h_bytes);

int32_t mdx_join_build(const void *d_keys, const int64_t *d_payload, const int64_t *d_offsets,
                       int64_t n, int32_t P, int32_t key_type, void *d_table_mem,
                       size_t table_bytes, mdx_table *h_table, int32_t *d_status,
                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Join probe: inner equi-join of a partitioned probe (right) table against a
 * built table, partition by partition.
 *
 * Section V-B ("cuDF Merge"): the probe half of the worker's merge; the
 * figure's "fraction match" is the share of right rows whose key occurs on
 * the left.
 * Output rows are (key, left payload, right payload), one per pair of equal-
 * key rows (multiset semantics).  Partition p's output rows occupy
 * [d_out_offsets[p], d_out_offsets[p+1]); d_out_offsets [P+1] int64 is always
 * written and d_out_offsets[P] is the total |J|.  Within a partition the row
 * order is implementation-defined (compare after sorting).
 * If |J| > out_capacity, rows that would land at or past out_capacity are
 * not written, the output contents are unspecified, and
 * MDX_DEV_OUTPUT_OVERFLOW is set; d_out_offsets is still exact, so a caller
 * can size the output and call again.  out_capacity == 0 with NULL output
 * pointers computes d_out_offsets only.
 * Arguments: d_keys [n] (the table's key type), d_payload [n], d_offsets
 * [P+1] of the probe table; d_ws of at least mdx_join_probe_workspace_bytes(
 * n, P, key_type) bytes; d_out_key [out_capacity] (key type), d_out_lpay and
 * d_out_rpay [out_capacity] int64.
 * A probe row whose destination differs from the partition its offsets place
 * it in finds no match and is reported with MDX_DEV_BAD_PARTITIONING.
 * ------------------------------------------------------------------------- */
int32_t mdx_join_probe_workspace_bytes(int64_t n_probe, int32_t P, int32_t key_type,
                                       size_t *h_bytes);

int32_t mdx_join_probe(const mdx_table *h_table, const void *d_keys, const int64_t *d_payload,
                       const int64_t *d_offsets, int64_t n, void *d_ws, size_t ws_bytes,
                       void *d_out_key, int64_t *d_out_lpay, int64_t *d_out_rpay,
                       int64_t out_capacity, int64_t *d_out_offsets, int32_t *d_status,
                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Join count: the per-partition output counts of the inner join of two
 * partitioned tables, without materializing it.
 *
 * Section V-B ("cuDF Merge"): the size of every partition's merge output,
 * sum over keys k of (build rows with key k) x (probe rows with key k) --
 * what a worker needs to size its output, and all that can be computed when
 * the output is too large to hold (heavily repeated keys).  The build keys
 * are counted per distinct key into a hash table in the workspace (rows are
 * first aggregated per workgroup, so a key repeated millions of times costs
 * one global update per workgroup), then every probe key looks up its
 * count.  Nothing is kept for later probes: the table lives in d_ws.
 * Arguments: d_lkeys [n_build] and d_lofs [P+1] (a table partitioned by
 * mdx_hash_partition), d_rkeys [n_probe] and d_rofs [P+1] likewise, both of
 * key_type; d_ws of at least mdx_join_count_workspace_bytes(n_build,
 * n_probe, P, key_type) bytes; d_out_offsets [P+1] int64 receives exactly
 * what mdx_join_probe writes there (exclusive prefix of the per-partition
 * counts, total in d_out_offsets[P]).  A row whose destination differs from
 * the partition its offsets place it in is skipped and reported with
 * MDX_DEV_BAD_PARTITIONING.
 * ------------------------------------------------------------------------- */
int32_t mdx_join_count_workspace_bytes(int64_t n_build, int64_t n_probe, int32_t P,
                                       int32_t key_type, size_t *h_bytes);

int32_t mdx_join_count(const void *d_lkeys, const int64_t *d_lofs, int64_t n_build,
                       const void *d_rkeys, const int64_t *d_rofs, int64_t n_probe, int32_t P,
                       int32_t key_type, void *d_ws, size_t ws_bytes, int64_t *d_out_offsets,
                       int32_t *d_status, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Merge: the whole per-worker path in one call.
 *
 * Section V-B ("cuDF Merge") with Section IV-B's buffers: the hash shuffle's
 * local partition of both frames followed by the merge of every partition,
 * on raw device buffers (no serialization, as the paper's point-to-point
 * layer sends them).
 * Partitions the left (build) and right (probe) tables into P destinations,
 * then joins every partition.  Inside the workspace each destination's rows
 * are further split by the top bits of the hash into sub-buckets small
 * enough for one workgroup's LDS, and every sub-bucket is joined in LDS
 * (a radix join).  If a build sub-bucket is too large for LDS (heavily
 * repeated keys), the device switches to the global-table join of
 * mdx_join_build/mdx_join_probe instead; no host synchronization is needed
 * for that choice.  Output exactly as mdx_join_probe (partition p at
 * [d_out_offsets[p], d_out_offsets[p+1]), total in d_out_offsets[P],
 * MDX_DEV_OUTPUT_OVERFLOW if out_capacity is too small; row order inside a
 * partition is implementation-defined).
 * d_ws: at least mdx_merge_workspace_bytes(nL, nR, P, key_type) bytes.
 * ------------------------------------------------------------------------- */
int32_t mdx_merge_workspace_bytes(int64_t n_left, int64_t n_right, int32_t P, int32_t key_type,
                                  size_t *h_bytes);

int32_t mdx_merge(const void *d_left_keys, const int64_t *d_left_payload, int64_t n_left,
                  const void *d_right_keys, const int64_t *d_right_payload, int64_t n_right,
                  int32_t key_type, int32_t P, void *d_ws, size_t ws_bytes, void *d_out_key,
                  int64_t *d_out_lpay, int64_t *d_out_rpay, int64_t out_capacity,
                  int64_t *d_out_offsets, int32_t *d_status, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched merges: many independent merges in one call.
 *
 * A worker of the paper's benchmark merges every frame it holds (Section
 * V-B); a service that answers many merge requests has many such merges at
 * once, most of them small.  One small merge alone leaves the device idle
 * between its dependent launches; a batch keeps several in flight.
 *
 * Merge i of h_descs[0..count) computes exactly what mdx_merge computes
 * with the same arguments (same output rows, same offsets, same device
 * status bits); merges are independent and may differ in sizes, key type
 * and P.  As in fused batches (below), a build sub-bucket too large for an
 * LDS table is joined in table-sized chunks rather than by the global-table
 * join, so a merge of a batch makes no launches for that join.  The merges run on up to `lanes` concurrent lanes: HIP streams the
 * library creates at the default priority on first use on a device and
 * keeps until the process ends.  The lanes are forked from `stream` and
 * joined back to it with events, so the batch is ordered on `stream` like a
 * single call and can be captured into a HIP graph.  Merges are assigned
 * largest first (by n_left + n_right), each to the lane with the fewest rows
 * so far (ties: the lowest lane); a lane runs its merges one after another
 * in its own slice of d_ws, sized for its largest merge.  With lanes = 1,
 * or a single merge, everything runs on `stream` itself.
 *
 * h_descs: host array, read during the call only.  lanes: 1..MDX_MAX_LANES.
 * d_ws: at least mdx_merge_batch_workspace_bytes(count, h_descs, lanes)
 * bytes (depends on the sizes, key types and P of the merges only).
 * Errors: MDX_ERR_INVALID for count < 0, a null h_descs with count > 0,
 * lanes out of range, or any descriptor mdx_merge would reject (the
 * message names the merge's index); MDX_ERR_WORKSPACE for a short
 * workspace.  Nothing is enqueued on an error.  Outputs of different merges
 * must not overlap one another.
 * ------------------------------------------------------------------------- */
#define MDX_MAX_LANES 8

typedef struct mdx_merge_desc {
    const void *d_left_keys;        /* [n_left] build keys, key_type */
    const int64_t *d_left_payload;  /* [n_left] */
    int64_t n_left;
    const void *d_right_keys;       /* [n_right] probe keys, key_type */
    const int64_t *d_right_payload; /* [n_right] */
    int64_t n_right;
    int32_t key_type; /* MDX_KEY_I32 or MDX_KEY_I64, both tables */
    int32_t P;        /* partitions, 1..MDX_MAX_P */
    void *d_out_key;  /* [out_capacity] output columns, as mdx_merge */
    int64_t *d_out_lpay;
    int64_t *d_out_rpay;
    int64_t out_capacity;
    int64_t *d_out_offsets; /* [P+1] */
    int32_t *d_status;      /* may be NULL; may be shared by merges */
} mdx_merge_desc;

int32_t mdx_merge_batch_workspace_bytes(int32_t count, const mdx_merge_desc *h_descs,
                                        int32_t lanes, size_t *h_bytes);

int32_t mdx_merge_batch(int32_t count, const mdx_merge_desc *h_descs, int32_t lanes, void *d_ws,
                        size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Fused batches: every step of many merges in one launch per step.
 *
 * For the same workload as mdx_merge_batch (Section V-B: a worker, or a
 * service, with many merges of uneven sizes at once).  Instead of running
 * whole merges side by side, a batch runs each step of the merge -- first
 * partition pass, segmented pass, LDS join, output offsets -- once for all
 * merges: one kernel launch per step covers every merge's tiles (merge m
 * owns a range of the launch's workgroups, found from a prefix of the
 * merges' block counts), and the join's workgroups take sub-buckets of all
 * merges from one ticket counter.  A batch of thousands of merges is then
 * about a dozen launches per wave instead of twenty per merge.
 *
 * Merge i computes the rows and offsets mdx_merge computes with the same
 * descriptor (row order inside a partition is implementation-defined, as
 * there), with one difference of method: a build sub-bucket too large for a
 * workgroup's LDS table (heavily repeated keys) is joined in table-sized
 * chunks by its workgroup instead of by the global-table join, so a batch
 * never leaves the radix join.  That is exact for any input but slow when a
 * few keys repeat very many times; mdx_merge handles such inputs better.
 *
 * Tuning (h_tuning: NULL, or one entry per merge): `fill` is the average
 * build rows of a sub-bucket as a fraction of an LDS table (0: 0.9; else in
 * [0.05, 1]); `fanout` caps the first pass's destinations (0: 128; else in
 * [1, 4096]); `part_rows` picks the first pass's rows per thread, 2 or 8
 * (0: by destinations; 8 needs at most 256 destinations, else 2 is used);
 * `reserved` must be 0.  Tuning changes speed only, never results.
 *
 * Workspace: merges are packed, largest first within each key width, into
 * waves whose workspace fits d_ws; waves run one after another.
 * mdx_batch_workspace_bytes gives the least workspace that runs the batch
 * (*h_min_bytes, waves of one merge at the worst) and the workspace that
 * runs it as one wave (*h_all_bytes).
 *
 * mdx_batch_create checks every descriptor as mdx_merge would and plans the
 * batch for d_ws (which must stay allocated and unused by others while the
 * batch exists): the plan's device records are written into pinned host
 * memory the batch owns (the one allocation here: host memory, none on the
 * device).  mdx_batch_run enqueues on `stream` the copy of those records
 * into d_ws followed by the launches; it can be captured into a HIP graph,
 * whose replays then need the batch, d_ws and every merge's buffers alive
 * and unchanged.  Runs of one batch must be ordered (they share d_ws).
 * mdx_batch_info reports the waves and kernel launches of one run.
 * mdx_batch_destroy waits until the last run enqueued outside a capture has
 * copied the records, then frees them; the caller destroys no batch whose
 * graph may still be replayed.
 * Errors: MDX_ERR_INVALID for count < 0, a null h_descs with count > 0,
 * bad tuning, a descriptor mdx_merge would reject (the message names the
 * merge); MDX_ERR_WORKSPACE when d_ws is smaller than *h_min_bytes;
 * MDX_ERR_HIP when the pinned allocation fails.
 * ------------------------------------------------------------------------- */
typedef struct mdx_batch_tuning {
    float fill;
    int32_t fanout;
    int32_t part_rows;
    int32_t reserved;
} mdx_batch_tuning;

typedef struct mdx_batch mdx_batch;

int32_t mdx_batch_workspace_bytes(int32_t count, const mdx_merge_desc *h_descs,
                                  const mdx_batch_tuning *h_tuning, size_t *h_min_bytes,
                                  size_t *h_all_bytes);

int32_t mdx_batch_create(int32_t count, const mdx_merge_desc *h_descs,
                         const mdx_batch_tuning *h_tuning, void *d_ws, size_t ws_bytes,
                         mdx_batch **h_batch);

int32_t mdx_batch_info(const mdx_batch *batch, int32_t *h_waves, int32_t *h_launches);

int32_t mdx_batch_run(mdx_batch *batch, hipStream_t stream);

int32_t mdx_batch_destroy(mdx_batch *batch);

/* ---------------------------------------------------------------------------
 * Serving: merge requests admitted as slots and memory free up.
 *
 * For a service that answers a stream of merge requests (each one a merge of
 * Section V-B): a server owns `slots` slots, each a HIP stream (created at
 * the default priority), a completion event and a slice of d_ws sized for
 * the largest merge it accepts (n_left <= max_left, n_right <= max_right,
 * P <= max_P, either key type).  mdx_server_submit admits a merge into a
 * free slot if the bytes of the merges in flight plus this one's -- inputs
 * and outputs: (n_left + n_right)(key bytes + 8) + out_capacity (key bytes
 * + 16) + 8 (P + 1) -- stay within budget_bytes; otherwise it returns
 * MDX_BUSY and enqueues nothing.  Merges in different slots run
 * concurrently and overlap on the device; each computes exactly what
 * mdx_merge computes with the same arguments (and, as a batch does, joins
 * a build sub-bucket too large for an LDS table in table-sized chunks).
 * mdx_server_poll returns the tags of merges that have finished (their
 * outputs are complete and visible to any stream) and frees their slots
 * and budget.  `ready`, if not
 * NULL, is an event the merge waits for before reading its inputs.
 *
 * A server is used from one host thread at a time.  The caller keeps d_ws
 * and every submitted merge's buffers alive until the merge is polled or
 * the server destroyed; mdx_server_destroy waits for merges in flight and
 * releases the streams and events.  Errors: MDX_ERR_INVALID for slots
 * outside [1, MDX_MAX_SLOTS], bad limits, a descriptor mdx_merge would
 * reject, a merge beyond the limits or larger than the whole budget;
 * MDX_ERR_WORKSPACE for a short workspace; MDX_ERR_HIP for runtime
 * failures.
 * ------------------------------------------------------------------------- */
#define MDX_MAX_SLOTS 32

typedef struct mdx_server mdx_server;

int32_t mdx_server_workspace_bytes(int32_t slots, int64_t max_left, int64_t max_right,
                                   int32_t max_P, size_t *h_bytes);

int32_t mdx_server_create(int32_t slots, int64_t max_left, int64_t max_right, int32_t max_P,
                          size_t budget_bytes, void *d_ws, size_t ws_bytes,
                          mdx_server **h_server);

int32_t mdx_server_submit(mdx_server *server, const mdx_merge_desc *h_desc, int64_t tag,
                          hipEvent_t ready, int32_t *h_slot);

/* A probe of a device-resident build table (built once with mdx_join_build),
 * admitted like a merge: for a service that keeps its build tables on the
 * device and answers many probe requests against them (each one the join
 * step of Section V-B's merge, without rebuilding the left table).  The probe
 * rows (any order) are partitioned by the table's P in the slot's workspace,
 * then probed with the global-table probe; the outputs are exactly those of
 * mdx_hash_partition + mdx_join_probe with the same arguments.  The request
 * holds n (key bytes + 8) + out_capacity (key bytes + 16) + 8 (P + 1) bytes
 * of the budget.  The caller keeps the table (h_table and its memory) and the
 * probe's buffers alive and unchanged until the probe is polled.  Errors as
 * mdx_server_submit, and MDX_ERR_INVALID for a table built by another ABI
 * version, n > max_right or the table's P > max_P. */
typedef struct mdx_probe_desc {
    const void *d_keys;        /* [n] probe keys, the table's key type */
    const int64_t *d_payload;  /* [n] */
    int64_t n;
    void *d_out_key;           /* [out_capacity] output columns, as mdx_join_probe */
    int64_t *d_out_lpay;
    int64_t *d_out_rpay;
    int64_t out_capacity;
    int64_t *d_out_offsets;    /* [P+1] */
    int32_t *d_status;         /* may be NULL */
} mdx_probe_desc;

int32_t mdx_server_submit_probe(mdx_server *server, const mdx_table *h_table,
                                const mdx_probe_desc *h_desc, int64_t tag, hipEvent_t ready,
                                int32_t *h_slot);

int32_t mdx_server_poll(mdx_server *server, int64_t *h_tags, int32_t capacity,
                        int32_t *h_count);

/* Busy slots and bytes in flight (host-side bookkeeping; no device call). */
int32_t mdx_server_stats(const mdx_server *server, int32_t *h_busy_slots,
                         size_t *h_bytes_in_flight);

int32_t mdx_server_destroy(mdx_server *server);

/* ---------------------------------------------------------------------------
 * Sum of a matrix and its transpose (the paper's other benchmark, Section
 * V-B "Sum of cuPy Array and its Transpose": y = x + x.T on a chunked cuPy
 * array).
 *
 * y = x + x^T for an n x n row-major float64 matrix: y[i][j] is the IEEE-754
 * sum (round to nearest, ties to even) of x[i][j] and x[j][i], so the
 * result is the same bit for bit on any device.  d_y may equal d_x (in
 * place); otherwise the two must not overlap.  n = 0 is valid and enqueues
 * nothing.  Errors: MDX_ERR_INVALID for n outside [0, MDX_MAX_TRANSPOSE_N],
 * a null or misaligned matrix with n > 0, or a partial overlap.
 * ------------------------------------------------------------------------- */
#define MDX_MAX_TRANSPOSE_N (INT64_C(1) << 17) /* 137 GB; the grid of tile pairs fits a dispatch */

int32_t mdx_transpose_sum(const double *d_x, double *d_y, int64_t n, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Kernel timing for benchmarks.
 *
 * Brackets every launch of the named kernel, made by libmdx calls on the
 * calling thread, with hipEventRecord(h_starts[i], stream) before and
 * hipEventRecord(h_stops[i], stream) after, on the stream the kernel is
 * launched on, for i = *h_count; then increments *h_count.  Launches past
 * `capacity` are not bracketed (*h_count still counts them).  The caller
 * creates and destroys the events and keeps the arrays and the counter
 * alive while tracing.  Up to 16 kernels can be traced at once; kernel ==
 * NULL stops all tracing on the thread.  Names: "part_hist", "part_scatter",
 * "seg_hist", "seg_scatter", "rj_join", "tbl_init", "tbl_insert",
 * "grp_count", "grp_alloc", "grp_scatter", "probe_chain", "probe_expand",
 * "transpose_sum".
 * ------------------------------------------------------------------------- */
int32_t mdx_trace_kernel(const char *kernel, hipEvent_t *h_starts, hipEvent_t *h_stops,
                         int32_t capacity, int32_t *h_count);

#ifdef __cplusplus
}
#endif

#endif /* MDX_H */
