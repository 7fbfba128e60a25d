// The extern "C" entry points of libmdx: argument validation (pure host code,
// before anything is enqueued), workspace and table carving, and the order of
// kernel launches.  No device memory is allocated here.
#include <atomic>
#include <string>

#include "mdx.h"
#include "mdx_internal.hpp"

using namespace mdx;

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int32_t hip_fail(hipError_t e, const char *where)
{
    return fail(MDX_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool key_ok(int32_t kt)
{
    return kt == MDX_KEY_I32 || kt == MDX_KEY_I64;
}

bool aligned(const void *p, size_t a)
{
    return ((uintptr_t)p % a) == 0;
}

bool overlap(const void *a, size_t an, const void *b, size_t bn)
{
    if (!a || !b || an == 0 || bn == 0)
        return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bn && y < x + an;
}

int32_t check_sizes(int64_t n, int32_t P, int32_t key_type, const char *what)
{
    if (n < 0 || n > MDX_MAX_ROWS)
        return fail(MDX_ERR_INVALID, std::string(what) + ": row count out of range");
    if (P < 1 || P > MDX_MAX_P)
        return fail(MDX_ERR_INVALID, std::string(what) + ": P outside [1, MDX_MAX_P]");
    if (!key_ok(key_type))
        return fail(MDX_ERR_INVALID, std::string(what) + ": key_type must be MDX_KEY_I32 or MDX_KEY_I64");
    return MDX_OK;
}

// Columns of a table: keys (key_type wide) and int64 payloads.
int32_t check_columns(const void *keys, const int64_t *pay, int64_t n, int32_t kt,
                      const char *what)
{
    if (n > 0 && (!keys || !pay))
        return fail(MDX_ERR_INVALID, std::string(what) + ": null column with n > 0");
    if (!aligned(keys, (size_t)kt) || !aligned(pay, 8))
        return fail(MDX_ERR_INVALID, std::string(what) + ": misaligned column");
    return MDX_OK;
}

std::atomic<int> g_cu_count[64];

struct Trace {
    std::string kernel;
    hipEvent_t *starts = nullptr, *stops = nullptr;
    int32_t cap = 0;
    int32_t *count = nullptr;
};
constexpr int kMaxTraces = 8;
thread_local Trace g_trace[kMaxTraces];
thread_local int g_ntrace = 0;

Trace *find_trace(const char *kernel)
{
    for (int i = 0; i < g_ntrace; ++i)
        if (g_trace[i].kernel == kernel)
            return &g_trace[i];
    return nullptr;
}

}  // namespace

void mdx::trace_begin(const char *kernel, hipStream_t s)
{
    if (g_ntrace == 0)
        return;
    Trace *t = find_trace(kernel);
    if (t && *t->count < t->cap)
        (void)hipEventRecord(t->starts[*t->count], s);
}

void mdx::trace_end(const char *kernel, hipStream_t s)
{
    if (g_ntrace == 0)
        return;
    Trace *t = find_trace(kernel);
    if (!t)
        return;
    if (*t->count < t->cap)
        (void)hipEventRecord(t->stops[*t->count], s);
    ++*t->count;
}

int mdx::device_fill_blocks()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 1024;
    int cu = g_cu_count[dev].load(std::memory_order_relaxed);
    if (cu <= 0) {
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cu <= 0)
            cu = 256;
        g_cu_count[dev].store(cu, std::memory_order_relaxed);
    }
    return cu * 8;
}

extern "C" {

int32_t mdx_abi_version(void)
{
    return MDX_ABI_VERSION;
}

const char *mdx_status_string(int32_t status)
{
    switch (status) {
    case MDX_OK:
        return "ok";
    case MDX_ERR_INVALID:
        return "invalid argument";
    case MDX_ERR_WORKSPACE:
        return "workspace or table too small";
    case MDX_ERR_HIP:
        return "HIP runtime error";
    default:
        return "unknown status";
    }
}

const char *mdx_last_error(void)
{
    return g_err.c_str();
}

int32_t mdx_trace_kernel(const char *kernel, hipEvent_t *h_starts, hipEvent_t *h_stops,
                         int32_t capacity, int32_t *h_count)
{
    g_err.clear();
    if (!kernel) {
        for (int i = 0; i < kMaxTraces; ++i)
            g_trace[i] = Trace();
        g_ntrace = 0;
        return MDX_OK;
    }
    static const char *known[] = {"part_hist", "part_scatter", "tbl_init",
                                  "tbl_insert", "probe_chain", "probe_expand"};
    bool ok = false;
    for (const char *k : known)
        ok |= std::string(k) == kernel;
    if (!ok)
        return fail(MDX_ERR_INVALID, std::string("mdx_trace_kernel: unknown kernel ") + kernel);
    if (capacity < 0 || !h_count || (capacity > 0 && (!h_starts || !h_stops)))
        return fail(MDX_ERR_INVALID, "mdx_trace_kernel: bad event arrays or counter");
    Trace *t = find_trace(kernel);
    if (!t) {
        if (g_ntrace == kMaxTraces)
            return fail(MDX_ERR_INVALID, "mdx_trace_kernel: too many traced kernels");
        t = &g_trace[g_ntrace++];
    }
    t->kernel = kernel;
    t->starts = h_starts;
    t->stops = h_stops;
    t->cap = capacity;
    t->count = h_count;
    return MDX_OK;
}

// ---- partition ---------------------------------------------------------------

int32_t mdx_hash_partition_workspace_bytes(int64_t n, int32_t P, int32_t key_type, size_t *h_bytes)
{
    g_err.clear();
    if (int32_t e = check_sizes(n, P, key_type, "mdx_hash_partition_workspace_bytes"))
        return e;
    if (!h_bytes)
        return fail(MDX_ERR_INVALID, "mdx_hash_partition_workspace_bytes: h_bytes is null");
    *h_bytes = part_layout(n, P).bytes;
    return MDX_OK;
}

int32_t mdx_hash_partition(const void *d_keys, const int64_t *d_payload, int64_t n,
                           int32_t key_type, int32_t P, void *d_keys_out, int64_t *d_payload_out,
                           int64_t *d_offsets, void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_hash_partition";
    if (int32_t e = check_sizes(n, P, key_type, W))
        return e;
    if (int32_t e = check_columns(d_keys, d_payload, n, key_type, W))
        return e;
    if (int32_t e = check_columns(d_keys_out, d_payload_out, n, key_type, W))
        return e;
    if (!d_offsets || !aligned(d_offsets, 8))
        return fail(MDX_ERR_INVALID, "mdx_hash_partition: d_offsets null or misaligned");
    const size_t kb = (size_t)n * key_type, vb = (size_t)n * 8;
    if (overlap(d_keys, kb, d_keys_out, kb) || overlap(d_keys, kb, d_payload_out, vb) ||
        overlap(d_payload, vb, d_keys_out, kb) || overlap(d_payload, vb, d_payload_out, vb) ||
        overlap(d_keys_out, kb, d_payload_out, vb))
        return fail(MDX_ERR_INVALID, "mdx_hash_partition: output columns overlap inputs or each other");
    const PartLayout L = part_layout(n, P);
    if (!d_ws || !aligned(d_ws, kAlign))
        return fail(MDX_ERR_INVALID, "mdx_hash_partition: workspace null or not 256-byte aligned");
    if (ws_bytes < L.bytes)
        return fail(MDX_ERR_WORKSPACE, "mdx_hash_partition: workspace needs " +
                                           std::to_string(L.bytes) + " bytes");
    hipError_t e = launch_partition(d_keys, d_payload, n, key_type, P, d_keys_out, d_payload_out,
                                    d_offsets, d_ws, stream);
    return e == hipSuccess ? MDX_OK : hip_fail(e, W);
}

// ---- build ---------------------------------------------------------------------

int32_t mdx_join_table_bytes(int64_t n_build, int32_t P, int32_t key_type, size_t *h_bytes)
{
    g_err.clear();
    if (int32_t e = check_sizes(n_build, P, key_type, "mdx_join_table_bytes"))
        return e;
    if (!h_bytes)
        return fail(MDX_ERR_INVALID, "mdx_join_table_bytes: h_bytes is null");
    *h_bytes = table_layout(n_build, P).bytes;
    return MDX_OK;
}

static TView make_view(const mdx_table &t, const int64_t *off, int32_t pb, int32_t pe)
{
    TView v;
    v.slots = t.d_slots;
    v.gstart = t.d_gstart;
    v.grouped = t.d_grouped;
    v.off = off;
    v.flags = t.d_flags;
    v.bump = t.d_bump;
    v.pb = pb;
    v.pe = pe;
    v.d = make_dest(t.P);
    return v;
}

static mdx_table carve_table(void *mem, size_t bytes, int64_t n, int32_t P, int32_t key_type)
{
    const TableLayout L = table_layout(n, P);
    char *b = (char *)mem;
    mdx_table t;
    t.abi_version = MDX_ABI_VERSION;
    t.P = P;
    t.key_type = key_type;
    t.reserved = 0;
    t.n = n;
    t.d_mem = mem;
    t.bytes = bytes;
    t.d_offsets = (int64_t *)(b + L.off_off);
    t.d_flags = (int32_t *)(b + L.flags_off);
    t.d_bump = (int64_t *)(b + L.bump_off);
    t.d_slots = (uint64_t *)(b + L.slots_off);
    t.d_gstart = (int64_t *)(b + L.gstart_off);
    t.d_grouped = (int64_t *)(b + L.grouped_off);
    return t;
}

int32_t mdx_join_build(const void *d_keys, const int64_t *d_payload, const int64_t *d_offsets,
                       int64_t n, int32_t P, int32_t key_type, void *d_table_mem,
                       size_t table_bytes, mdx_table *h_table, int32_t *d_status,
                       hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_join_build";
    if (int32_t e = check_sizes(n, P, key_type, W))
        return e;
    if (int32_t e = check_columns(d_keys, d_payload, n, key_type, W))
        return e;
    if (!d_offsets || !aligned(d_offsets, 8))
        return fail(MDX_ERR_INVALID, "mdx_join_build: d_offsets null or misaligned");
    if (!h_table)
        return fail(MDX_ERR_INVALID, "mdx_join_build: h_table is null");
    if (!aligned(d_status, 4))
        return fail(MDX_ERR_INVALID, "mdx_join_build: d_status misaligned");
    const TableLayout L = table_layout(n, P);
    if (!d_table_mem || !aligned(d_table_mem, kAlign))
        return fail(MDX_ERR_INVALID, "mdx_join_build: table memory null or not 256-byte aligned");
    if (table_bytes < L.bytes)
        return fail(MDX_ERR_WORKSPACE,
                    "mdx_join_build: table needs " + std::to_string(L.bytes) + " bytes");
    const size_t kb = (size_t)n * key_type, vb = (size_t)n * 8;
    if (overlap(d_table_mem, table_bytes, d_keys, kb) ||
        overlap(d_table_mem, table_bytes, d_payload, vb) ||
        overlap(d_table_mem, table_bytes, d_offsets, (size_t)(P + 1) * 8))
        return fail(MDX_ERR_INVALID, "mdx_join_build: table memory overlaps the input");
    mdx_table t = carve_table(d_table_mem, table_bytes, n, P, key_type);
    hipError_t e = launch_table_setup(d_offsets, n, t.d_offsets, t.d_flags, t.d_bump, P, stream);
    if (e != hipSuccess)
        return hip_fail(e, W);
    e = launch_build(d_keys, d_payload, key_type, make_view(t, t.d_offsets, 0, P), d_status, stream);
    if (e != hipSuccess)
        return hip_fail(e, W);
    *h_table = t;
    return MDX_OK;
}

// ---- probe ---------------------------------------------------------------------

int32_t mdx_join_probe_workspace_bytes(int64_t n_probe, int32_t P, int32_t key_type,
                                       size_t *h_bytes)
{
    g_err.clear();
    if (int32_t e = check_sizes(n_probe, P, key_type, "mdx_join_probe_workspace_bytes"))
        return e;
    if (!h_bytes)
        return fail(MDX_ERR_INVALID, "mdx_join_probe_workspace_bytes: h_bytes is null");
    *h_bytes = probe_layout(n_probe, P).bytes;
    return MDX_OK;
}

static int32_t check_outputs(void *ok, int64_t *ol, int64_t *orr, int64_t cap, int32_t kt,
                             int64_t *d_out_offsets, int32_t *d_status, const char *W)
{
    if (cap < 0)
        return fail(MDX_ERR_INVALID, std::string(W) + ": out_capacity < 0");
    if (cap > 0 && (!ok || !ol || !orr))
        return fail(MDX_ERR_INVALID, std::string(W) + ": null output column with out_capacity > 0");
    if (!aligned(ok, (size_t)kt) || !aligned(ol, 8) || !aligned(orr, 8))
        return fail(MDX_ERR_INVALID, std::string(W) + ": misaligned output column");
    if (!d_out_offsets || !aligned(d_out_offsets, 8))
        return fail(MDX_ERR_INVALID, std::string(W) + ": d_out_offsets null or misaligned");
    if (!aligned(d_status, 4))
        return fail(MDX_ERR_INVALID, std::string(W) + ": d_status misaligned");
    const size_t kb = (size_t)cap * kt, vb = (size_t)cap * 8;
    if (overlap(ok, kb, ol, vb) || overlap(ok, kb, orr, vb) || overlap(ol, vb, orr, vb))
        return fail(MDX_ERR_INVALID, std::string(W) + ": output columns overlap");
    return MDX_OK;
}

int32_t mdx_join_probe(const mdx_table *h_table, const void *d_keys, const int64_t *d_payload,
                       const int64_t *d_offsets, int64_t n, void *d_ws, size_t ws_bytes,
                       void *d_out_key, int64_t *d_out_lpay, int64_t *d_out_rpay,
                       int64_t out_capacity, int64_t *d_out_offsets, int32_t *d_status,
                       hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_join_probe";
    if (!h_table || h_table->abi_version != MDX_ABI_VERSION || !h_table->d_slots)
        return fail(MDX_ERR_INVALID, "mdx_join_probe: table missing or built by another ABI version");
    const mdx_table &t = *h_table;
    const int32_t P = t.P, kt = t.key_type;
    if (int32_t e = check_sizes(n, P, kt, W))
        return e;
    if (int32_t e = check_columns(d_keys, d_payload, n, kt, W))
        return e;
    if (!d_offsets || !aligned(d_offsets, 8))
        return fail(MDX_ERR_INVALID, "mdx_join_probe: d_offsets null or misaligned");
    if (int32_t e = check_outputs(d_out_key, d_out_lpay, d_out_rpay, out_capacity, kt, d_out_offsets,
                                  d_status, W))
        return e;
    const ProbeLayout L = probe_layout(n, P);
    if (!d_ws || !aligned(d_ws, kAlign))
        return fail(MDX_ERR_INVALID, "mdx_join_probe: workspace null or not 256-byte aligned");
    if (ws_bytes < L.bytes)
        return fail(MDX_ERR_WORKSPACE,
                    "mdx_join_probe: workspace needs " + std::to_string(L.bytes) + " bytes");
    if (overlap(d_ws, ws_bytes, t.d_mem, t.bytes))
        return fail(MDX_ERR_INVALID, "mdx_join_probe: workspace overlaps the table");
    const ProbeWs w = probe_ws(d_ws, L);
    ProbeOut o;
    o.key = d_out_key;
    o.lpay = d_out_lpay;
    o.rpay = d_out_rpay;
    o.cap = out_capacity;
    o.offsets = d_out_offsets;
    hipError_t e = launch_probe_plan(d_offsets, n, P, w, stream);
    if (e == hipSuccess)
        e = launch_probe_group(d_keys, d_payload, kt, P, make_view(t, t.d_offsets, 0, P), 0, w, o,
                               d_status, stream);
    if (e == hipSuccess)
        e = launch_probe_finalize(P, w, o, stream);
    return e == hipSuccess ? MDX_OK : hip_fail(e, W);
}

// ---- merge -----------------------------------------------------------------------

namespace {

struct MergeLayout {
    PartLayout pl, pr;
    TableLayout tl;
    ProbeLayout ql;
    size_t partL_off, partR_off, lk_off, lv_off, offL_off, rk_off, rv_off, offR_off, table_off,
        probe_off, bytes;
};

MergeLayout merge_layout(int64_t nL, int64_t nR, int32_t P, int32_t kt)
{
    MergeLayout M;
    M.pl = part_layout(nL, P);
    M.pr = part_layout(nR, P);
    M.tl = table_layout(nL, P);
    M.ql = probe_layout(nR, P);
    size_t o = 0;
    M.partL_off = o;
    o += align_up(M.pl.bytes);
    M.partR_off = o;
    o += align_up(M.pr.bytes);
    M.lk_off = o;
    o += align_up((size_t)(nL > 0 ? nL : 1) * kt);
    M.lv_off = o;
    o += align_up((size_t)(nL > 0 ? nL : 1) * 8);
    M.offL_off = o;
    o += align_up((size_t)(P + 1) * 8);
    M.rk_off = o;
    o += align_up((size_t)(nR > 0 ? nR : 1) * kt);
    M.rv_off = o;
    o += align_up((size_t)(nR > 0 ? nR : 1) * 8);
    M.offR_off = o;
    o += align_up((size_t)(P + 1) * 8);
    M.table_off = o;
    o += align_up(M.tl.bytes);
    M.probe_off = o;
    o += align_up(M.ql.bytes);
    M.bytes = o;
    return M;
}

// Partitions per group: a group's tables (2 slots of 16 bytes per build
// row) should stay resident in the last-level cache while it is probed.
int32_t auto_group(int64_t nL, int32_t P)
{
    const double per_part = (2.0 * (double)nL / P + 16.0) * 16.0;
    const double target = 128.0 * 1024 * 1024;
    int32_t g = (int32_t)(target / per_part);
    if (g < 1)
        g = 1;
    if (g > P)
        g = P;
    return g;
}

}  // namespace

int32_t mdx_merge_workspace_bytes(int64_t n_left, int64_t n_right, int32_t P, int32_t key_type,
                                  size_t *h_bytes)
{
    g_err.clear();
    if (int32_t e = check_sizes(n_left, P, key_type, "mdx_merge_workspace_bytes"))
        return e;
    if (int32_t e = check_sizes(n_right, P, key_type, "mdx_merge_workspace_bytes"))
        return e;
    if (!h_bytes)
        return fail(MDX_ERR_INVALID, "mdx_merge_workspace_bytes: h_bytes is null");
    *h_bytes = merge_layout(n_left, n_right, P, key_type).bytes;
    return MDX_OK;
}

int32_t mdx_merge(const void *d_left_keys, const int64_t *d_left_payload, int64_t n_left,
                  const void *d_right_keys, const int64_t *d_right_payload, int64_t n_right,
                  int32_t key_type, int32_t P, void *d_ws, size_t ws_bytes, void *d_out_key,
                  int64_t *d_out_lpay, int64_t *d_out_rpay, int64_t out_capacity,
                  int64_t *d_out_offsets, int32_t *d_status, int32_t group_partitions,
                  hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_merge";
    if (int32_t e = check_sizes(n_left, P, key_type, W))
        return e;
    if (int32_t e = check_sizes(n_right, P, key_type, W))
        return e;
    if (int32_t e = check_columns(d_left_keys, d_left_payload, n_left, key_type, W))
        return e;
    if (int32_t e = check_columns(d_right_keys, d_right_payload, n_right, key_type, W))
        return e;
    if (int32_t e = check_outputs(d_out_key, d_out_lpay, d_out_rpay, out_capacity, key_type,
                                  d_out_offsets, d_status, W))
        return e;
    if (group_partitions < 0)
        return fail(MDX_ERR_INVALID, "mdx_merge: group_partitions < 0");
    const MergeLayout M = merge_layout(n_left, n_right, P, key_type);
    if (!d_ws || !aligned(d_ws, kAlign))
        return fail(MDX_ERR_INVALID, "mdx_merge: workspace null or not 256-byte aligned");
    if (ws_bytes < M.bytes)
        return fail(MDX_ERR_WORKSPACE,
                    "mdx_merge: workspace needs " + std::to_string(M.bytes) + " bytes");
    const size_t ob = (size_t)out_capacity * 8;
    if (overlap(d_ws, ws_bytes, d_out_key, (size_t)out_capacity * key_type) ||
        overlap(d_ws, ws_bytes, d_out_lpay, ob) || overlap(d_ws, ws_bytes, d_out_rpay, ob))
        return fail(MDX_ERR_INVALID, "mdx_merge: workspace overlaps the output");

    char *b = (char *)d_ws;
    void *lk = b + M.lk_off, *rk = b + M.rk_off;
    int64_t *lv = (int64_t *)(b + M.lv_off), *rv = (int64_t *)(b + M.rv_off);
    int64_t *offL = (int64_t *)(b + M.offL_off), *offR = (int64_t *)(b + M.offR_off);

    hipError_t e = launch_partition(d_left_keys, d_left_payload, n_left, key_type, P, lk, lv, offL,
                                    b + M.partL_off, stream);
    if (e == hipSuccess)
        e = launch_partition(d_right_keys, d_right_payload, n_right, key_type, P, rk, rv, offR,
                             b + M.partR_off, stream);
    if (e != hipSuccess)
        return hip_fail(e, W);

    mdx_table t = carve_table(b + M.table_off, M.tl.bytes, n_left, P, key_type);
    const ProbeWs w = probe_ws(b + M.probe_off, M.ql);
    ProbeOut o;
    o.key = d_out_key;
    o.lpay = d_out_lpay;
    o.rpay = d_out_rpay;
    o.cap = out_capacity;
    o.offsets = d_out_offsets;
    e = launch_table_setup(nullptr, 0, nullptr, t.d_flags, t.d_bump, P, stream);
    if (e == hipSuccess)
        e = launch_probe_plan(offR, n_right, P, w, stream);
    const int32_t gsz = group_partitions > 0 ? (group_partitions < P ? group_partitions : P)
                                             : auto_group(n_left, P);
    int group = 0;
    for (int32_t pb = 0; pb < P && e == hipSuccess; pb += gsz, ++group) {
        const int32_t pe = pb + gsz < P ? pb + gsz : P;
        // Every group reuses the start of the table region.
        const TView v = make_view(t, offL, pb, pe);
        e = launch_build(lk, lv, key_type, v, d_status, stream);
        if (e == hipSuccess)
            e = launch_probe_group(rk, rv, key_type, P, v, group, w, o, d_status, stream);
    }
    if (e == hipSuccess)
        e = launch_probe_finalize(P, w, o, stream);
    return e == hipSuccess ? MDX_OK : hip_fail(e, W);
}

}  // extern "C"
