// The extern "C" entry points of libmdx: argument validation (pure host code,
// before anything is enqueued), workspace and table carving, and the order of
// kernel launches.  No device memory is allocated here.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

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
constexpr int kMaxTraces = 16;
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
    case MDX_BUSY:
        return "busy: no free slot or memory budget (nothing enqueued)";
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
    static const char *known[] = {"part_hist",  "part_scatter", "tbl_init",    "tbl_insert",
                                  "probe_chain", "probe_expand", "seg_hist",    "seg_scatter",
                                  "rj_join",    "cnt_insert",   "cnt_probe",   "grp_count",
                                  "grp_alloc",  "grp_scatter",  "transpose_sum"};
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

}  // extern "C"

// Host checks of a partition call's columns and offsets (W names the caller).
static int32_t check_partition(const void *d_keys, const int64_t *d_payload, int64_t n,
                               int32_t key_type, int32_t P, const void *d_keys_out,
                               const int64_t *d_payload_out, const int64_t *d_offsets,
                               const char *W)
{
    if (int32_t e = check_sizes(n, P, key_type, W))
        return e;
    if (int32_t e = check_columns(d_keys, d_payload, n, key_type, W))
        return e;
    if (int32_t e = check_columns(d_keys_out, d_payload_out, n, key_type, W))
        return e;
    if (!d_offsets || !aligned(d_offsets, 8))
        return fail(MDX_ERR_INVALID, std::string(W) + ": d_offsets null or misaligned");
    const size_t kb = (size_t)n * key_type, vb = (size_t)n * 8;
    if (overlap(d_keys, kb, d_keys_out, kb) || overlap(d_keys, kb, d_payload_out, vb) ||
        overlap(d_payload, vb, d_keys_out, kb) || overlap(d_payload, vb, d_payload_out, vb) ||
        overlap(d_keys_out, kb, d_payload_out, vb))
        return fail(MDX_ERR_INVALID,
                    std::string(W) + ": output columns overlap inputs or each other");
    return MDX_OK;
}

extern "C" {

int32_t mdx_hash_partition(const void *d_keys, const int64_t *d_payload, int64_t n,
                           int32_t key_type, int32_t P, void *d_keys_out, int64_t *d_payload_out,
                           int64_t *d_offsets, void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_hash_partition";
    if (int32_t e = check_partition(d_keys, d_payload, n, key_type, P, d_keys_out, d_payload_out,
                                    d_offsets, W))
        return e;
    const PartLayout L = part_layout(n, P);
    if (!d_ws || !aligned(d_ws, kAlign))
        return fail(MDX_ERR_INVALID, "mdx_hash_partition: workspace null or not 256-byte aligned");
    if (ws_bytes < L.bytes)
        return fail(MDX_ERR_WORKSPACE, "mdx_hash_partition: workspace needs " +
                                           std::to_string(L.bytes) + " bytes");
    const PartArgs t = {d_keys, d_payload, n, d_keys_out, d_payload_out, d_offsets, nullptr, d_ws};
    hipError_t e = launch_partition(&t, 1, key_type, P, 0, 0, 0, stream);
    return e == hipSuccess ? MDX_OK : hip_fail(e, W);
}

}  // extern "C"

// ---- partition without allocation ---------------------------------------------------
// For callers that cannot allocate: the partition's workspace (per-(destination,
// tile) counts, destination totals; every entry is written before it is read, so
// nothing needs clearing) lives in this file-scope device array.  Every GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  In host code `scratch` names a host-side stand-in, not device memory:
// its device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address is passed to kernels.
namespace {

static __device__ __align__(256) unsigned char scratch[MDX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];

// Device address of the current device's scratch array (looked up on the first
// call on that device).
int32_t scratch_address(void **out, const char *W)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, W);
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MDX_ERR_INVALID, std::string(W) + ": device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(e, W);
        if (!p)
            return fail(MDX_ERR_HIP, std::string(W) + ": scratch array has no device address");
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return MDX_OK;
}

}  // namespace

extern "C" {

int32_t mdx_hash_partition_noalloc(const void *d_keys, const int64_t *d_payload, int64_t n,
                                   int32_t key_type, int32_t P, void *d_keys_out,
                                   int64_t *d_payload_out, int64_t *d_offsets,
                                   hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_hash_partition_noalloc";
    if (int32_t e = check_partition(d_keys, d_payload, n, key_type, P, d_keys_out, d_payload_out,
                                    d_offsets, W))
        return e;
    const PartLayout L = part_layout(n, P);
    if (L.bytes > (size_t)MDX_NOALLOC_SCRATCH_BYTES)
        return fail(MDX_ERR_WORKSPACE,
                    std::string(W) + ": needs " + std::to_string(L.bytes) +
                        " bytes of scratch, more than the library's " +
                        std::to_string((size_t)MDX_NOALLOC_SCRATCH_BYTES) +
                        "; call mdx_hash_partition with a workspace instead");
    void *ws = nullptr;
    if (int32_t e = scratch_address(&ws, W))
        return e;
    const PartArgs t = {d_keys, d_payload, n, d_keys_out, d_payload_out, d_offsets, nullptr, ws};
    hipError_t e = launch_partition(&t, 1, key_type, P, 0, 0, 0, stream);
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
    v.skip = nullptr;
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
    e = launch_build(d_keys, d_payload, key_type, make_view(t, t.d_offsets, 0, P), n, d_status, 0,
                     stream);
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
    hipError_t e = launch_probe_plan(d_offsets, n, P, w, nullptr, stream);
    if (e == hipSuccess)
        e = launch_probe_group(d_keys, d_payload, kt, P, make_view(t, t.d_offsets, 0, P), 0, w, o,
                               d_status, 0, stream);
    if (e == hipSuccess)
        e = launch_probe_finalize(P, w, o, nullptr, stream);
    return e == hipSuccess ? MDX_OK : hip_fail(e, W);
}

// ---- count-only join ---------------------------------------------------------------

namespace {

// d_ws of mdx_join_count: sanitized build and probe offsets, per-partition
// counts, then the count table's slots.
struct CountLayout {
    int64_t nslots;
    size_t off_off, offp_off, pcount_off, slots_off, bytes;
};

CountLayout count_layout(int64_t n_build, int32_t P)
{
    CountLayout L;
    L.nslots = 2 * n_build + 16 * (int64_t)P;
    size_t o = 0;
    L.off_off = o;
    o += align_up((size_t)(P + 1) * 8);
    L.offp_off = o;
    o += align_up((size_t)(P + 1) * 8);
    L.pcount_off = o;
    o += align_up((size_t)P * 8);
    L.slots_off = o;
    o += align_up((size_t)L.nslots * 16);
    L.bytes = o;
    return L;
}

int32_t check_keys(const void *keys, const int64_t *ofs, int64_t n, int32_t kt, const char *W,
                   const char *side)
{
    if (n > 0 && !keys)
        return fail(MDX_ERR_INVALID, std::string(W) + ": null " + side + " keys with n > 0");
    if (!aligned(keys, (size_t)kt))
        return fail(MDX_ERR_INVALID, std::string(W) + ": misaligned " + side + " keys");
    if (!ofs || !aligned(ofs, 8))
        return fail(MDX_ERR_INVALID, std::string(W) + ": " + side + " offsets null or misaligned");
    return MDX_OK;
}

}  // namespace

int32_t mdx_join_count_workspace_bytes(int64_t n_build, int64_t n_probe, int32_t P,
                                       int32_t key_type, size_t *h_bytes)
{
    g_err.clear();
    const char *W = "mdx_join_count_workspace_bytes";
    if (int32_t e = check_sizes(n_build, P, key_type, W))
        return e;
    if (int32_t e = check_sizes(n_probe, P, key_type, W))
        return e;
    if (!h_bytes)
        return fail(MDX_ERR_INVALID, std::string(W) + ": h_bytes is null");
    *h_bytes = count_layout(n_build, P).bytes;
    return MDX_OK;
}

int32_t mdx_join_count(const void *d_lkeys, const int64_t *d_lofs, int64_t n_build,
                       const void *d_rkeys, const int64_t *d_rofs, int64_t n_probe, int32_t P,
                       int32_t key_type, void *d_ws, size_t ws_bytes, int64_t *d_out_offsets,
                       int32_t *d_status, hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_join_count";
    if (int32_t e = check_sizes(n_build, P, key_type, W))
        return e;
    if (int32_t e = check_sizes(n_probe, P, key_type, W))
        return e;
    if (int32_t e = check_keys(d_lkeys, d_lofs, n_build, key_type, W, "build"))
        return e;
    if (int32_t e = check_keys(d_rkeys, d_rofs, n_probe, key_type, W, "probe"))
        return e;
    if (!d_out_offsets || !aligned(d_out_offsets, 8))
        return fail(MDX_ERR_INVALID, std::string(W) + ": d_out_offsets null or misaligned");
    if (!aligned(d_status, 4))
        return fail(MDX_ERR_INVALID, std::string(W) + ": d_status misaligned");
    const CountLayout L = count_layout(n_build, P);
    if (!d_ws || !aligned(d_ws, kAlign))
        return fail(MDX_ERR_INVALID, std::string(W) + ": workspace null or not 256-byte aligned");
    if (ws_bytes < L.bytes)
        return fail(MDX_ERR_WORKSPACE,
                    std::string(W) + ": workspace needs " + std::to_string(L.bytes) + " bytes");
    if (overlap(d_ws, ws_bytes, d_out_offsets, (size_t)(P + 1) * 8))
        return fail(MDX_ERR_INVALID, std::string(W) + ": workspace overlaps d_out_offsets");
    char *b = (char *)d_ws;
    TView v = {};
    v.slots = (uint64_t *)(b + L.slots_off);
    v.off = (const int64_t *)(b + L.off_off);
    v.pb = 0;
    v.pe = P;
    v.d = make_dest(P);
    const hipError_t e = launch_join_count(d_lkeys, d_lofs, n_build, d_rkeys, d_rofs, n_probe,
                                           key_type, v, (int64_t *)(b + L.offp_off),
                                           (uint64_t *)(b + L.pcount_off), d_out_offsets,
                                           d_status, stream);
    return e == hipSuccess ? MDX_OK : hip_fail(e, W);
}

// ---- merge -----------------------------------------------------------------------

namespace {

// How mdx_merge splits partitions into sub-buckets for the radix join: each
// partition into Q = 2^qbits sub-buckets by the top hash bits, sized so that
// an average sub-bucket of the larger side fills ~80% of an LDS table: the
// build side's rows must fit the table, and the probe side's should fit one
// probe batch (with sub-buckets sized by a small build side alone, a large
// probe side would leave a few workgroups looping over many batches each).
// The first pass partitions by (p, top q1bits) with a fan-out of at most 128
// (long, coalesced output runs); the segmented second pass splits each of
// those buckets by the next q2bits (at most 256 ways).
struct MergePlan {
    int qbits, q1bits, q2bits;
};

// fill: average rows of the larger side per sub-bucket, as a fraction of a
// table of `cap` rows (the join's table: the fused batch's holds more rows);
// fanout: the first pass's largest number of destinations.
MergePlan merge_plan(int64_t nL, int64_t nR, int32_t P, double fill = kJoinFill, int fanout = 128,
                     int cap = kJoinCap)
{
    MergePlan m;
    const double per = fill * cap;
    const double want = (double)std::max(nL, nR) / ((double)P * per);
    m.qbits = want <= 1.0 ? 0 : ceil_log2((int64_t)(want + 0.999999));
    // keep the sub-bucket count bounded; oversized sub-buckets fall back to
    // the global-table join
    while (m.qbits > 0 && ((int64_t)P << m.qbits) > (int64_t)1 << 22)
        --m.qbits;
    for (;; --m.qbits) {
        m.q1bits = 0;
        while (m.q1bits < m.qbits && ((int64_t)P << (m.q1bits + 1)) <= fanout)
            ++m.q1bits;
        m.q2bits = m.qbits - m.q1bits;
        while (m.q2bits > 8) {  // the segmented pass splits at most 256 ways
            ++m.q1bits;
            --m.q2bits;
        }
        // the first pass handles at most MDX_MAX_P destinations
        if (m.qbits == 0 || ((int64_t)P << m.q1bits) <= MDX_MAX_P)
            break;
    }
    return m;
}

struct MergeLayout {
    MergePlan plan;
    int64_t nA, S;  // first-pass destinations, sub-buckets
    PartLayout pl, pr;
    SegLayout sl, sr;
    RJoinLayout jl;
    TableLayout tl;
    ProbeLayout ql;
    size_t partL_off, partR_off, lk1_off, lv1_off, rk1_off, rv1_off, offAL_off, offAR_off,
        offPL_off, offPR_off, digL_off, digR_off, segL_off, segR_off, lk2_off, lv2_off, rk2_off,
        rv2_off, subL_off, subR_off, rjoin_off, table_off, probe_off, bytes;
};

// chunked: the merge joins oversized build sub-buckets in chunks and has no
// global-table join (no table or probe workspace).
MergeLayout merge_layout(int64_t nL, int64_t nR, int32_t P, int32_t kt, bool chunked = false)
{
    MergeLayout M;
    M.plan = merge_plan(nL, nR, P);
    M.nA = (int64_t)P << M.plan.q1bits;
    M.S = (int64_t)P << M.plan.qbits;
    M.pl = part_layout(nL, (int32_t)M.nA);
    M.pr = part_layout(nR, (int32_t)M.nA);
    M.sl = seg_layout(nL, M.nA, M.plan.q2bits);
    M.sr = seg_layout(nR, M.nA, M.plan.q2bits);
    M.jl = rjoin_layout(P, M.plan.qbits);
    M.tl = table_layout(nL, P);
    M.ql = probe_layout(nR, P);
    const size_t kL = (size_t)(nL > 0 ? nL : 1), kR = (size_t)(nR > 0 ? nR : 1);
    const bool two = M.plan.q2bits > 0;
    size_t o = 0;
    auto take = [&](size_t &field, size_t bytes) {
        field = o;
        o += align_up(bytes);
    };
    take(M.partL_off, M.pl.bytes);
    take(M.partR_off, M.pr.bytes);
    take(M.lk1_off, kL * kt);
    take(M.lv1_off, kL * 8);
    take(M.rk1_off, kR * kt);
    take(M.rv1_off, kR * 8);
    take(M.offAL_off, (size_t)(M.nA + 1) * 8);
    take(M.offAR_off, (size_t)(M.nA + 1) * 8);
    take(M.offPL_off, (size_t)(P + 1) * 8);
    take(M.offPR_off, (size_t)(P + 1) * 8);
    take(M.digL_off, two ? kL + 4 : 0);  // + 4: read as 4-byte words
    take(M.digR_off, two ? kR + 4 : 0);
    take(M.segL_off, two ? M.sl.bytes : 0);
    take(M.segR_off, two ? M.sr.bytes : 0);
    take(M.lk2_off, two ? kL * kt : 0);
    take(M.lv2_off, two ? kL * 8 : 0);
    take(M.rk2_off, two ? kR * kt : 0);
    take(M.rv2_off, two ? kR * 8 : 0);
    take(M.subL_off, two ? (size_t)(M.S + 1) * 8 : 0);
    take(M.subR_off, two ? (size_t)(M.S + 1) * 8 : 0);
    take(M.rjoin_off, M.jl.bytes);
    take(M.table_off, chunked ? 0 : M.tl.bytes);
    take(M.probe_off, chunked ? 0 : M.ql.bytes);
    M.bytes = o;
    return M;
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

// Host checks of one merge's arguments (W names the caller in messages).
static int32_t check_merge(const mdx_merge_desc &d, const char *W)
{
    if (int32_t e = check_sizes(d.n_left, d.P, d.key_type, W))
        return e;
    if (int32_t e = check_sizes(d.n_right, d.P, d.key_type, W))
        return e;
    if (int32_t e = check_columns(d.d_left_keys, d.d_left_payload, d.n_left, d.key_type, W))
        return e;
    if (int32_t e = check_columns(d.d_right_keys, d.d_right_payload, d.n_right, d.key_type, W))
        return e;
    return check_outputs(d.d_out_key, d.d_out_lpay, d.d_out_rpay, d.out_capacity, d.key_type,
                         d.d_out_offsets, d.d_status, W);
}

// Checks of a merge's workspace [ws, ws + ws_bytes) against its layout.
static int32_t check_merge_ws(const mdx_merge_desc &d, const void *ws, size_t ws_bytes,
                              size_t need, const char *W)
{
    if (!ws || !aligned(ws, kAlign))
        return fail(MDX_ERR_INVALID, std::string(W) + ": workspace null or not 256-byte aligned");
    if (ws_bytes < need)
        return fail(MDX_ERR_WORKSPACE,
                    std::string(W) + ": workspace needs " + std::to_string(need) + " bytes");
    const size_t ob = (size_t)d.out_capacity * 8;
    if (overlap(ws, ws_bytes, d.d_out_key, (size_t)d.out_capacity * d.key_type) ||
        overlap(ws, ws_bytes, d.d_out_lpay, ob) || overlap(ws, ws_bytes, d.d_out_rpay, ob))
        return fail(MDX_ERR_INVALID, std::string(W) + ": workspace overlaps the output");
    return MDX_OK;
}

// Enqueue one checked merge on `stream`, workspace at d_ws (its layout
// merge_layout(..., chunked)).  chunked: oversized build sub-buckets are
// joined in LDS chunks, so the global-table join's launches are left out.
static hipError_t enqueue_merge(const mdx_merge_desc &d, void *d_ws, hipStream_t stream,
                                bool chunked = false)
{
    const int32_t P = d.P, key_type = d.key_type;
    const int64_t n_left = d.n_left, n_right = d.n_right;
    const MergeLayout M = merge_layout(n_left, n_right, P, key_type, chunked);
    char *b = (char *)d_ws;
    const MergePlan &pl = M.plan;
    const int nA = (int)M.nA;
    void *lk1 = b + M.lk1_off, *rk1 = b + M.rk1_off;
    int64_t *lv1 = (int64_t *)(b + M.lv1_off), *rv1 = (int64_t *)(b + M.rv1_off);
    int64_t *offAL = (int64_t *)(b + M.offAL_off), *offAR = (int64_t *)(b + M.offAR_off);
    int32_t *d_status = d.d_status;
    ProbeOut o;
    o.key = d.d_out_key;
    o.lpay = d.d_out_lpay;
    o.rpay = d.d_out_rpay;
    o.cap = d.out_capacity;
    o.offsets = d.d_out_offsets;

    // 1. partition both tables by (partition, top q1bits of the hash); with a
    // second pass, every output row's next q2bits go beside it as a byte
    const bool two = pl.q2bits > 0;
    uint8_t *digL = two ? (uint8_t *)(b + M.digL_off) : nullptr;
    uint8_t *digR = two ? (uint8_t *)(b + M.digR_off) : nullptr;
    const PartArgs pt[2] = {
        {d.d_left_keys, d.d_left_payload, n_left, lk1, lv1, offAL, digL, b + M.partL_off},
        {d.d_right_keys, d.d_right_payload, n_right, rk1, rv1, offAR, digR, b + M.partR_off}};
    hipError_t e = launch_partition(pt, 2, key_type, P, pl.q1bits, pl.q1bits, pl.q2bits, stream);

    // 2. split every first-pass bucket by the next q2bits: sub-buckets
    const void *lk = lk1, *rk = rk1;
    const int64_t *lv = lv1, *rv = rv1, *subL = offAL, *subR = offAR;
    if (two && e == hipSuccess) {
        void *lk2 = b + M.lk2_off, *rk2 = b + M.rk2_off;
        int64_t *lv2 = (int64_t *)(b + M.lv2_off), *rv2 = (int64_t *)(b + M.rv2_off);
        int64_t *sL = (int64_t *)(b + M.subL_off), *sR = (int64_t *)(b + M.subR_off);
        const SegArgs st[2] = {{lk1, lv1, digL, n_left, offAL, lk2, lv2, sL, b + M.segL_off},
                               {rk1, rv1, digR, n_right, offAR, rk2, rv2, sR, b + M.segR_off}};
        e = launch_seg_partition(st, 2, key_type, nA, pl.q1bits, pl.q2bits, stream);
        lk = lk2;
        rk = rk2;
        lv = lv2;
        rv = rv2;
        subL = sL;
        subR = sR;
    }

    // 3. radix join of every sub-bucket in LDS, if every build sub-bucket fits
    const RJoinWs jw = rjoin_ws(b + M.rjoin_off, M.jl);
    if (e == hipSuccess)
        e = launch_rjoin_plan(subL, subR, M.S, jw, chunked, stream);
    if (e == hipSuccess)
        e = launch_rjoin(lk, lv, subL, rk, rv, subR, key_type, P, pl.qbits, jw, o, d_status,
                         chunked, stream);

    // 4. otherwise (a sub-bucket too large for LDS: heavy key repetition),
    // the global-table join over the first-pass output; its kernels do
    // nothing when the radix join ran.  No sub-bucket can exceed the table
    // when the whole build side fits it: then they are not launched.
    if (chunked || n_left <= kJoinCap) {
        if (e == hipSuccess)
            e = launch_merge_finalize(P, pl.qbits, jw, nullptr, o, stream);
        return e;
    }
    int64_t *offPL = (int64_t *)(b + M.offPL_off), *offPR = (int64_t *)(b + M.offPR_off);
    mdx_table t = carve_table(b + M.table_off, M.tl.bytes, n_left, P, key_type);
    const ProbeWs w = probe_ws(b + M.probe_off, M.ql);
    if (e == hipSuccess)
        e = launch_fallback_setup(offAL, offAR, 1 << pl.q1bits, P, n_left, n_right, offPL, offPR,
                                  t.d_offsets, t.d_flags, t.d_bump, w, jw.use, stream);
    TView v = make_view(t, t.d_offsets, 0, P);
    v.skip = jw.use;
    // grids sized to the rows (~16K per workgroup): these launches mostly
    // return at once, and return sooner with fewer workgroups
    auto blocks = [](int64_t rows) { return (int)std::min<int64_t>((rows >> 14) + 1, 1 << 20); };
    if (e == hipSuccess)
        e = launch_build(lk1, lv1, key_type, v, n_left, d_status, blocks(n_left), stream);
    if (e == hipSuccess)
        e = launch_probe_group(rk1, rv1, key_type, P, v, 0, w, o, d_status, blocks(n_right),
                               stream);
    if (e == hipSuccess)
        e = launch_merge_finalize(P, pl.qbits, jw, &w, o, stream);
    return e;
}

int32_t mdx_merge(const void *d_left_keys, const int64_t *d_left_payload, int64_t n_left,
                  const void *d_right_keys, const int64_t *d_right_payload, int64_t n_right,
                  int32_t key_type, int32_t P, void *d_ws, size_t ws_bytes, void *d_out_key,
                  int64_t *d_out_lpay, int64_t *d_out_rpay, int64_t out_capacity,
                  int64_t *d_out_offsets, int32_t *d_status, hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_merge";
    const mdx_merge_desc d = {d_left_keys,   d_left_payload, n_left,       d_right_keys,
                              d_right_payload, n_right,      key_type,     P,
                              d_out_key,     d_out_lpay,     d_out_rpay,   out_capacity,
                              d_out_offsets, d_status};
    if (int32_t e = check_merge(d, W))
        return e;
    if (int32_t e = check_merge_ws(d, d_ws, ws_bytes, merge_layout(n_left, n_right, P, key_type).bytes, W))
        return e;
    const hipError_t e = enqueue_merge(d, d_ws, stream);
    return e == hipSuccess ? MDX_OK : hip_fail(e, W);
}

// ---- batched merges ----------------------------------------------------------------

}  // extern "C"

namespace {

// Lane of every merge (largest first, each to the lane with the fewest rows
// so far; ties to the lowest lane), the order merges are enqueued in, and
// every lane's workspace slice (sized for its largest merge).
struct BatchPlan {
    std::vector<int32_t> order, lane;
    std::vector<size_t> lane_off;
    int32_t used = 0;
    size_t bytes = 0;
};

BatchPlan batch_plan(int32_t count, const mdx_merge_desc *h, int32_t lanes)
{
    BatchPlan B;
    B.order.resize((size_t)count);
    B.lane.assign((size_t)count, 0);
    for (int32_t i = 0; i < count; ++i)
        B.order[(size_t)i] = i;
    std::stable_sort(B.order.begin(), B.order.end(), [&](int32_t a, int32_t b) {
        return h[a].n_left + h[a].n_right > h[b].n_left + h[b].n_right;
    });
    const int32_t L = count < lanes ? (count > 0 ? count : 1) : lanes;
    std::vector<int64_t> load((size_t)L, 0);
    std::vector<size_t> need((size_t)L, 0);
    for (int32_t i : B.order) {
        int32_t l = 0;
        for (int32_t k = 1; k < L; ++k)
            if (load[(size_t)k] < load[(size_t)l])
                l = k;
        B.lane[(size_t)i] = l;
        load[(size_t)l] += h[i].n_left + h[i].n_right;
        const size_t b =
            merge_layout(h[i].n_left, h[i].n_right, h[i].P, h[i].key_type, true).bytes;
        need[(size_t)l] = need[(size_t)l] > b ? need[(size_t)l] : b;
    }
    B.used = L;
    B.lane_off.resize((size_t)L);
    size_t o = 0;
    for (int32_t l = 0; l < L; ++l) {
        B.lane_off[(size_t)l] = o;
        o += align_up(need[(size_t)l]);
    }
    B.bytes = o;
    return B;
}

// Lane streams: created once per device, kept until the process ends.
std::mutex g_lane_mu;
std::vector<std::vector<hipStream_t>> g_lane_streams;

hipError_t lane_streams(int32_t n, hipStream_t *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lock(g_lane_mu);
    if ((int)g_lane_streams.size() <= dev)
        g_lane_streams.resize((size_t)dev + 1);
    auto &v = g_lane_streams[(size_t)dev];
    while ((int32_t)v.size() < n) {
        hipStream_t s;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess)
            return e;
        v.push_back(s);
    }
    for (int32_t l = 0; l < n; ++l)
        out[l] = v[(size_t)l];
    return hipSuccess;
}

int32_t check_batch(int32_t count, const mdx_merge_desc *h, int32_t lanes, const char *W)
{
    if (count < 0)
        return fail(MDX_ERR_INVALID, std::string(W) + ": count < 0");
    if (count > 0 && !h)
        return fail(MDX_ERR_INVALID, std::string(W) + ": h_descs is null");
    if (lanes < 1 || lanes > MDX_MAX_LANES)
        return fail(MDX_ERR_INVALID, std::string(W) + ": lanes outside [1, MDX_MAX_LANES]");
    for (int32_t i = 0; i < count; ++i) {
        const std::string Wi = std::string(W) + " (merge " + std::to_string(i) + ")";
        if (int32_t e = check_sizes(h[i].n_left, h[i].P, h[i].key_type, Wi.c_str()))
            return e;
        if (int32_t e = check_sizes(h[i].n_right, h[i].P, h[i].key_type, Wi.c_str()))
            return e;
    }
    return MDX_OK;
}

}  // namespace

extern "C" {

int32_t mdx_merge_batch_workspace_bytes(int32_t count, const mdx_merge_desc *h_descs,
                                        int32_t lanes, size_t *h_bytes)
{
    g_err.clear();
    const char *W = "mdx_merge_batch_workspace_bytes";
    if (int32_t e = check_batch(count, h_descs, lanes, W))
        return e;
    if (!h_bytes)
        return fail(MDX_ERR_INVALID, std::string(W) + ": h_bytes is null");
    *h_bytes = batch_plan(count, h_descs, lanes).bytes;
    return MDX_OK;
}

int32_t mdx_merge_batch(int32_t count, const mdx_merge_desc *h_descs, int32_t lanes, void *d_ws,
                        size_t ws_bytes, hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_merge_batch";
    if (int32_t e = check_batch(count, h_descs, lanes, W))
        return e;
    const BatchPlan B = batch_plan(count, h_descs, lanes);
    if (count > 0 && (!d_ws || !aligned(d_ws, kAlign)))
        return fail(MDX_ERR_INVALID, std::string(W) + ": workspace null or not 256-byte aligned");
    if (ws_bytes < B.bytes)
        return fail(MDX_ERR_WORKSPACE,
                    std::string(W) + ": workspace needs " + std::to_string(B.bytes) + " bytes");
    for (int32_t i = 0; i < count; ++i) {
        const mdx_merge_desc &d = h_descs[i];
        const std::string Wi = std::string(W) + " (merge " + std::to_string(i) + ")";
        if (int32_t e = check_merge(d, Wi.c_str()))
            return e;
        // its lane's slice holds its layout; its output stays clear of the
        // whole batch workspace
        const size_t need = merge_layout(d.n_left, d.n_right, d.P, d.key_type, true).bytes;
        if (int32_t e = check_merge_ws(d, (char *)d_ws + B.lane_off[(size_t)B.lane[(size_t)i]],
                                       need, need, Wi.c_str()))
            return e;
        if (int32_t e = check_merge_ws(d, d_ws, B.bytes, 0, Wi.c_str()))
            return e;
    }
    if (count == 0)
        return MDX_OK;

    // One lane: the caller's stream itself.  Otherwise fork the lanes from
    // `stream` and join them back with events.
    hipStream_t ls[MDX_MAX_LANES];
    hipError_t e = hipSuccess;
    if (B.used == 1) {
        ls[0] = stream;
    } else {
        e = lane_streams(B.used, ls);
        if (e != hipSuccess)
            return hip_fail(e, W);
    }
    hipEvent_t fork = nullptr, join[MDX_MAX_LANES] = {};
    if (B.used > 1) {
        e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventRecord(fork, stream);
        for (int32_t l = 0; l < B.used && e == hipSuccess; ++l)
            e = hipStreamWaitEvent(ls[l], fork, 0);
    }
    for (size_t k = 0; k < B.order.size() && e == hipSuccess; ++k) {
        const int32_t i = B.order[k], l = B.lane[(size_t)i];
        e = enqueue_merge(h_descs[i], (char *)d_ws + B.lane_off[(size_t)l], ls[l], true);
    }
    if (B.used > 1) {
        // join every lane that was forked, even after an error, so that
        // `stream` never runs ahead of work already enqueued on a lane
        for (int32_t l = 0; l < B.used; ++l) {
            hipError_t e2 = hipEventCreateWithFlags(&join[l], hipEventDisableTiming);
            if (e2 == hipSuccess)
                e2 = hipEventRecord(join[l], ls[l]);
            if (e2 == hipSuccess)
                e2 = hipStreamWaitEvent(stream, join[l], 0);
            if (e == hipSuccess)
                e = e2;
        }
        for (int32_t l = 0; l < B.used; ++l)
            if (join[l])
                (void)hipEventDestroy(join[l]);
        if (fork)
            (void)hipEventDestroy(fork);
    }
    return e == hipSuccess ? MDX_OK : hip_fail(e, W);
}

// ---- fused batches: one launch per step for all merges --------------------------------

}  // extern "C"

namespace {

// Per-unit block prefixes, one array of M + 1 entries per step.
enum BatchStep { kTiles, kScan, kOffs, kSegPlan, kSegHist, kSegScan, kSegTiles, kSubs, kSteps };
constexpr int64_t kUnitMaxBlocks = (int64_t)1 << 30;  // per step and unit (grid limit 2^31 - 1)

struct Tuned {
    double fill;
    int fanout, rows;
};

int32_t check_tuning(const mdx_batch_tuning *h, int32_t i, Tuned *out, const char *W)
{
    const mdx_batch_tuning t = h ? h[i] : mdx_batch_tuning{0.0f, 0, 0, 0};
    const std::string Wi = std::string(W) + " (merge " + std::to_string(i) + ")";
    if (t.reserved != 0)
        return fail(MDX_ERR_INVALID, Wi + ": tuning.reserved must be 0");
    if (!(t.fill == 0.0f || (t.fill >= 0.05f && t.fill <= 1.0f)))
        return fail(MDX_ERR_INVALID, Wi + ": tuning.fill outside {0} or [0.05, 1]");
    if (t.fanout < 0 || t.fanout > MDX_MAX_P)
        return fail(MDX_ERR_INVALID, Wi + ": tuning.fanout outside [0, MDX_MAX_P]");
    if (t.part_rows != 0 && t.part_rows != 2 && t.part_rows != 8)
        return fail(MDX_ERR_INVALID, Wi + ": tuning.part_rows not 0, 2 or 8");
    out->fill = t.fill == 0.0f ? kJoinFill : (double)t.fill;
    out->fanout = t.fanout ? t.fanout : 128;
    out->rows = t.part_rows;
    return MDX_OK;
}

// One merge of a fused batch: its plan and the layout of its workspace
// (offsets from `base`, its place in d_ws).
struct FusedMerge {
    int32_t idx = 0;
    MergePlan plan = {};
    int64_t nA = 0, S = 0;
    int R = 0, kt = 0, wave = 0;
    PartLayout pl = {}, pr = {};
    SegLayout sl = {}, sr = {};
    size_t partL = 0, partR = 0, lk1 = 0, lv1 = 0, rk1 = 0, rv1 = 0, offAL = 0, offAR = 0,
           digL = 0, digR = 0, segL = 0, segR = 0, lk2 = 0, lv2 = 0, rk2 = 0, rv2 = 0, subL = 0,
           subR = 0, jst = 0, jbase = 0, bytes = 0, base = 0;
    int64_t blocks[kSteps] = {};
};

FusedMerge fused_merge(const mdx_merge_desc &d, int32_t idx, const Tuned &t)
{
    FusedMerge F;
    F.idx = idx;
    F.kt = d.key_type;
    F.plan = merge_plan(d.n_left, d.n_right, d.P, t.fill, t.fanout, kBatchJoinCap);
    F.nA = (int64_t)d.P << F.plan.q1bits;
    F.S = (int64_t)d.P << F.plan.qbits;
    const int deflt = part_rows_per_thread((int32_t)F.nA);
    F.R = t.rows == 2 ? kPartRowsLarge
                      : (t.rows == 8 ? (F.nA <= kPartSmallMaxP ? kPartRowsSmall : kPartRowsLarge)
                                     : deflt);
    F.pl = part_layout(d.n_left, (int32_t)F.nA, F.R);
    F.pr = part_layout(d.n_right, (int32_t)F.nA, F.R);
    const bool two = F.plan.q2bits > 0;
    if (two) {
        F.sl = seg_layout(d.n_left, F.nA, F.plan.q2bits);
        F.sr = seg_layout(d.n_right, F.nA, F.plan.q2bits);
    }
    const size_t kL = (size_t)(d.n_left > 0 ? d.n_left : 1),
                 kR = (size_t)(d.n_right > 0 ? d.n_right : 1), kt = (size_t)d.key_type;
    size_t o = 0;
    auto take = [&](size_t &field, size_t bytes) {
        field = o;
        o += align_up(bytes);
    };
    take(F.partL, F.pl.bytes);
    take(F.partR, F.pr.bytes);
    take(F.lk1, kL * kt);
    take(F.lv1, kL * 8);
    take(F.rk1, kR * kt);
    take(F.rv1, kR * 8);
    take(F.offAL, (size_t)(F.nA + 1) * 8);
    take(F.offAR, (size_t)(F.nA + 1) * 8);
    take(F.digL, two ? kL + 4 : 0);
    take(F.digR, two ? kR + 4 : 0);
    take(F.segL, two ? F.sl.bytes : 0);
    take(F.segR, two ? F.sr.bytes : 0);
    take(F.lk2, two ? kL * kt : 0);
    take(F.lv2, two ? kL * 8 : 0);
    take(F.rk2, two ? kR * kt : 0);
    take(F.rv2, two ? kR * 8 : 0);
    take(F.subL, two ? (size_t)(F.S + 1) * 8 : 0);
    take(F.subR, two ? (size_t)(F.S + 1) * 8 : 0);
    take(F.jst, (size_t)F.S * 8);
    take(F.jbase, (size_t)F.S * 8);
    F.bytes = o;
    F.blocks[kTiles] = F.pl.ntiles + F.pr.ntiles;
    F.blocks[kScan] = (2 * F.nA + kWavesPerBlock - 1) / kWavesPerBlock;
    F.blocks[kOffs] = 2;
    F.blocks[kSegPlan] = two ? 2 : 0;
    F.blocks[kSegHist] = two ? F.sl.max_chunks + F.sr.max_chunks : 0;
    F.blocks[kSegScan] = two ? 2 * F.nA : 0;
    F.blocks[kSegTiles] = two ? F.sl.max_tiles + F.sr.max_tiles : 0;
    F.blocks[kSubs] = F.S;
    return F;
}

// Bytes of the records one merge adds to the plan image, and a bound on the
// image: records, block prefixes (M + 1 entries per step and unit) and the
// 16-byte alignment of every array, with at most one unit per merge.
size_t merge_record_bytes()
{
    return align_up(part_rec_bytes(), 16) + align_up(seg_rec_bytes(), 16) +
           align_up(sizeof(JoinRec), 16);
}

size_t image_bound(int32_t count)
{
    const size_t c = (size_t)count;
    return c * merge_record_bytes() + (size_t)kSteps * 4 * (2 * c) + c * (3 + kSteps) * 16;
}

// d_ws: [plan image][ticket per unit][waves]
size_t fixed_bytes(int32_t count)
{
    return align_up(image_bound(count)) + align_up((size_t)(count > 0 ? count : 1) * 4);
}

// Merges of one key width and tile shape within one wave.
struct BatchUnit {
    int kt = 0, R = 0, maxD = 1, maxbits = 0;
    bool dig = false;
    std::vector<int32_t> merges;  // indexes into the FusedMerge list
    int64_t total[kSteps] = {};
    size_t part_off = 0, seg_off = 0, join_off = 0, pre_off[kSteps] = {}, ticket_off = 0;
};

int32_t check_fused(int32_t count, const mdx_merge_desc *h, const mdx_batch_tuning *t,
                    std::vector<FusedMerge> *out, const char *W)
{
    if (count < 0)
        return fail(MDX_ERR_INVALID, std::string(W) + ": count < 0");
    if (count > 0 && !h)
        return fail(MDX_ERR_INVALID, std::string(W) + ": h_descs is null");
    out->clear();
    out->reserve((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        const std::string Wi = std::string(W) + " (merge " + std::to_string(i) + ")";
        if (int32_t e = check_sizes(h[i].n_left, h[i].P, h[i].key_type, Wi.c_str()))
            return e;
        if (int32_t e = check_sizes(h[i].n_right, h[i].P, h[i].key_type, Wi.c_str()))
            return e;
        Tuned tu;
        if (int32_t e = check_tuning(t, i, &tu, W))
            return e;
        out->push_back(fused_merge(h[i], i, tu));
    }
    return MDX_OK;
}

}  // namespace

struct mdx_batch {
    int device = 0;
    char *d_ws = nullptr;
    size_t image_bytes = 0;
    char *h_image = nullptr;   // pinned
    hipEvent_t copied = nullptr;  // after the last eager run's copy of h_image
    std::vector<BatchUnit> units;
    int32_t waves = 0, launches = 0;
};

extern "C" {

int32_t mdx_batch_workspace_bytes(int32_t count, const mdx_merge_desc *h_descs,
                                  const mdx_batch_tuning *h_tuning, size_t *h_min_bytes,
                                  size_t *h_all_bytes)
{
    g_err.clear();
    const char *W = "mdx_batch_workspace_bytes";
    std::vector<FusedMerge> F;
    if (int32_t e = check_fused(count, h_descs, h_tuning, &F, W))
        return e;
    if (!h_min_bytes || !h_all_bytes)
        return fail(MDX_ERR_INVALID, std::string(W) + ": null output pointer");
    size_t most = 0, all = 0;
    for (const FusedMerge &f : F) {
        most = std::max(most, align_up(f.bytes));
        all += align_up(f.bytes);
    }
    *h_min_bytes = fixed_bytes(count) + most;
    *h_all_bytes = fixed_bytes(count) + all;
    return MDX_OK;
}

int32_t mdx_batch_create(int32_t count, const mdx_merge_desc *h_descs,
                         const mdx_batch_tuning *h_tuning, void *d_ws, size_t ws_bytes,
                         mdx_batch **h_batch)
{
    g_err.clear();
    const char *W = "mdx_batch_create";
    if (!h_batch)
        return fail(MDX_ERR_INVALID, std::string(W) + ": h_batch is null");
    *h_batch = nullptr;
    std::vector<FusedMerge> F;
    if (int32_t e = check_fused(count, h_descs, h_tuning, &F, W))
        return e;
    if (!d_ws || !aligned(d_ws, kAlign))
        return fail(MDX_ERR_INVALID, std::string(W) + ": workspace null or not 256-byte aligned");
    const size_t fixed = fixed_bytes(count);
    size_t most = 0;
    for (const FusedMerge &f : F)
        most = std::max(most, align_up(f.bytes));
    if (ws_bytes < fixed + most)
        return fail(MDX_ERR_WORKSPACE,
                    std::string(W) + ": workspace needs at least " + std::to_string(fixed + most) +
                        " bytes");
    for (int32_t i = 0; i < count; ++i) {
        const std::string Wi = std::string(W) + " (merge " + std::to_string(i) + ")";
        if (int32_t e = check_merge(h_descs[i], Wi.c_str()))
            return e;
        if (int32_t e = check_merge_ws(h_descs[i], d_ws, ws_bytes, 0, Wi.c_str()))
            return e;
    }

    // Waves: merges of one key width and tile shape together, largest first;
    // a wave takes merges until the next does not fit.
    std::vector<int32_t> order((size_t)count);
    for (int32_t i = 0; i < count; ++i)
        order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const FusedMerge &x = F[(size_t)a], &y = F[(size_t)b];
        if (x.kt != y.kt)
            return x.kt > y.kt;
        if (x.R != y.R)
            return x.R > y.R;
        return x.bytes > y.bytes;
    });
    std::unique_ptr<mdx_batch> B(new mdx_batch);
    const size_t cap = ws_bytes - fixed;
    size_t used = 0;
    int wave = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        FusedMerge &f = F[(size_t)order[k]];
        const size_t b = align_up(f.bytes);
        if (k > 0 && used + b > cap) {
            ++wave;
            used = 0;
        }
        f.wave = wave;
        f.base = fixed + used;
        used += b;
        // a unit holds one key width and tile shape of one wave, within the
        // grid limits
        BatchUnit *u = B->units.empty() ? nullptr : &B->units.back();
        bool fresh = !u || u->kt != f.kt || u->R != f.R ||
                     F[(size_t)u->merges.back()].wave != f.wave;
        for (int st = 0; st < kSteps && !fresh; ++st)
            fresh = u->total[st] + f.blocks[st] > kUnitMaxBlocks;
        if (fresh) {
            B->units.emplace_back();
            u = &B->units.back();
            u->kt = f.kt;
            u->R = f.R;
        }
        u->merges.push_back(order[k]);
        for (int st = 0; st < kSteps; ++st)
            u->total[st] += f.blocks[st];
        u->maxD = std::max<int>(u->maxD, (int)f.nA);
        u->maxbits = std::max(u->maxbits, f.plan.q2bits);
        u->dig = u->dig || f.plan.q2bits > 0;
    }
    B->waves = count > 0 ? wave + 1 : 0;

    // The plan image: per unit its records and block prefixes.
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes, 16);
        return at;
    };
    const size_t tickets = align_up(image_bound(count));
    for (size_t ui = 0; ui < B->units.size(); ++ui) {
        BatchUnit &u = B->units[ui];
        const size_t M = u.merges.size();
        u.part_off = take(M * part_rec_bytes());
        u.seg_off = take(M * seg_rec_bytes());
        u.join_off = take(M * sizeof(JoinRec));
        for (int st = 0; st < kSteps; ++st)
            u.pre_off[st] = take((M + 1) * 4);
        u.ticket_off = tickets + ui * 4;
    }
    B->image_bytes = o;
    if (o > image_bound(count))
        return fail(MDX_ERR_INVALID, std::string(W) + ": internal plan size");  // cannot happen
    if (o > 0) {
        hipError_t e = hipHostMalloc((void **)&B->h_image, o, hipHostMallocDefault);
        if (e != hipSuccess)
            return hip_fail(e, W);
        memset(B->h_image, 0, o);
    }
    char *ws = (char *)d_ws;
    for (BatchUnit &u : B->units) {
        std::vector<uint32_t> pre[kSteps];
        for (int st = 0; st < kSteps; ++st)
            pre[st].assign(1, 0u);
        for (size_t j = 0; j < u.merges.size(); ++j) {
            const FusedMerge &f = F[(size_t)u.merges[j]];
            const mdx_merge_desc &d = h_descs[f.idx];
            char *b = ws + f.base;
            const bool two = f.plan.q2bits > 0;
            uint8_t *digL = two ? (uint8_t *)(b + f.digL) : nullptr;
            uint8_t *digR = two ? (uint8_t *)(b + f.digR) : nullptr;
            int64_t *offAL = (int64_t *)(b + f.offAL), *offAR = (int64_t *)(b + f.offAR);
            const PartArgs pt[2] = {
                {d.d_left_keys, d.d_left_payload, d.n_left, b + f.lk1, (int64_t *)(b + f.lv1),
                 offAL, digL, b + f.partL},
                {d.d_right_keys, d.d_right_payload, d.n_right, b + f.rk1, (int64_t *)(b + f.rv1),
                 offAR, digR, b + f.partR}};
            part_rec(pt, f.kt, d.P, f.plan.q1bits, f.R, f.plan.q1bits, f.plan.q2bits,
                     B->h_image + u.part_off + j * part_rec_bytes());
            JoinRec jr = {};
            if (two) {
                const SegArgs sa[2] = {
                    {b + f.lk1, (int64_t *)(b + f.lv1), digL, d.n_left, offAL, b + f.lk2,
                     (int64_t *)(b + f.lv2), (int64_t *)(b + f.subL), b + f.segL},
                    {b + f.rk1, (int64_t *)(b + f.rv1), digR, d.n_right, offAR, b + f.rk2,
                     (int64_t *)(b + f.rv2), (int64_t *)(b + f.subR), b + f.segR}};
                seg_rec(sa, f.kt, f.nA, f.plan.q1bits, f.plan.q2bits,
                        B->h_image + u.seg_off + j * seg_rec_bytes());
                jr.lk = b + f.lk2;
                jr.lv = (const int64_t *)(b + f.lv2);
                jr.subL = (const int64_t *)(b + f.subL);
                jr.rk = b + f.rk2;
                jr.rv = (const int64_t *)(b + f.rv2);
                jr.subR = (const int64_t *)(b + f.subR);
            } else {
                jr.lk = b + f.lk1;
                jr.lv = (const int64_t *)(b + f.lv1);
                jr.subL = offAL;
                jr.rk = b + f.rk1;
                jr.rv = (const int64_t *)(b + f.rv1);
                jr.subR = offAR;
            }
            jr.jstatus = (uint64_t *)(b + f.jst);
            jr.jbase = (int64_t *)(b + f.jbase);
            jr.S = f.S;
            jr.o.key = d.d_out_key;
            jr.o.lpay = d.d_out_lpay;
            jr.o.rpay = d.d_out_rpay;
            jr.o.cap = d.out_capacity;
            jr.o.offsets = d.d_out_offsets;
            jr.status = d.d_status;
            jr.P = d.P;
            jr.qbits = f.plan.qbits;
            jr.by_part = rjoin_by_partition(f.plan.qbits, rjoin_grid(u.total[kSubs])) ? 1 : 0;
            memcpy(B->h_image + u.join_off + j * sizeof(JoinRec), &jr, sizeof(jr));
            for (int st = 0; st < kSteps; ++st)
                pre[st].push_back(pre[st].back() + (uint32_t)f.blocks[st]);
        }
        for (int st = 0; st < kSteps; ++st)
            memcpy(B->h_image + u.pre_off[st], pre[st].data(), pre[st].size() * 4);
    }
    int launches = B->image_bytes > 0 ? 1 : 0;
    for (const BatchUnit &u : B->units)
        launches += 4 + (u.total[kSegPlan] > 0 ? 4 : 0) + 3;
    B->launches = launches;
    B->d_ws = ws;
    (void)hipGetDevice(&B->device);
    *h_batch = B.release();
    return MDX_OK;
}

int32_t mdx_batch_info(const mdx_batch *batch, int32_t *h_waves, int32_t *h_launches)
{
    g_err.clear();
    if (!batch || !h_waves || !h_launches)
        return fail(MDX_ERR_INVALID, "mdx_batch_info: null argument");
    *h_waves = batch->waves;
    *h_launches = batch->launches;
    return MDX_OK;
}

int32_t mdx_batch_run(mdx_batch *batch, hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_batch_run";
    if (!batch)
        return fail(MDX_ERR_INVALID, std::string(W) + ": batch is null");
    if (batch->units.empty())
        return MDX_OK;
    char *img = batch->d_ws;
    hipError_t e = hipMemcpyAsync(img, batch->h_image, batch->image_bytes, hipMemcpyHostToDevice,
                                  stream);
    // an eager run's copy reads the pinned image after this call returns:
    // mdx_batch_destroy waits for it (a captured run's copy belongs to its
    // graph, which the caller keeps the batch alive for)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (e == hipSuccess)
        e = hipStreamIsCapturing(stream, &cap);
    if (e == hipSuccess && cap == hipStreamCaptureStatusNone) {
        if (!batch->copied)
            e = hipEventCreateWithFlags(&batch->copied, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventRecord(batch->copied, stream);
    }
    for (const BatchUnit &u : batch->units) {
        if (e != hipSuccess)
            break;
        const int M = (int)u.merges.size();
        auto stage = [&](int st) {
            return BatchStage{(const uint32_t *)(img + u.pre_off[st]), (uint32_t)u.total[st]};
        };
        e = launch_partition_batch(img + u.part_off, M, u.kt, u.R, u.maxD, u.dig, stage(kTiles),
                                   stage(kScan), stage(kOffs), stream);
        if (e == hipSuccess && u.total[kSegPlan] > 0)
            e = launch_seg_batch(img + u.seg_off, M, u.kt, u.maxbits, stage(kSegPlan),
                                 stage(kSegHist), stage(kSegScan), stage(kSegTiles), stream);
        if (e == hipSuccess)
            e = launch_rjoin_batch((const JoinRec *)(img + u.join_off), M,
                                   (const uint32_t *)(img + u.pre_off[kSubs]),
                                   (uint32_t)u.total[kSubs], (uint32_t *)(img + u.ticket_off), u.kt,
                                   stream);
    }
    return e == hipSuccess ? MDX_OK : hip_fail(e, W);
}

int32_t mdx_batch_destroy(mdx_batch *batch)
{
    g_err.clear();
    if (!batch)
        return MDX_OK;
    hipError_t e = hipSuccess;
    if (batch->copied) {
        e = hipEventSynchronize(batch->copied);
        const hipError_t e2 = hipEventDestroy(batch->copied);
        e = e == hipSuccess ? e2 : e;
    }
    if (batch->h_image) {
        const hipError_t e2 = hipHostFree(batch->h_image);
        e = e == hipSuccess ? e2 : e;
    }
    delete batch;
    return e == hipSuccess ? MDX_OK : hip_fail(e, "mdx_batch_destroy");
}

// ---- serving: merges admitted as slots and memory free up ------------------------------

}  // extern "C"

struct mdx_server {
    int device = 0;
    int32_t slots = 0;
    int64_t max_left = 0, max_right = 0;
    int32_t max_P = 0;
    size_t budget = 0, in_flight = 0, slot_bytes = 0;
    char *d_ws = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;
    std::vector<int64_t> tag;       // tag of the merge in the slot
    std::vector<size_t> held;       // its bytes against the budget
    std::vector<char> busy;
};

namespace {

// Bytes a merge holds while it runs: its inputs and outputs.
size_t request_bytes(const mdx_merge_desc &d)
{
    const size_t row = (size_t)d.key_type + 8;
    return (size_t)d.n_left * row + (size_t)d.n_right * row +
           (size_t)d.out_capacity * ((size_t)d.key_type + 16) + (size_t)(d.P + 1) * 8;
}

// Bytes a probe against a resident table holds while it runs.
size_t probe_request_bytes(const mdx_probe_desc &d, int32_t P, int32_t key_type)
{
    return (size_t)d.n * ((size_t)key_type + 8) +
           (size_t)d.out_capacity * ((size_t)key_type + 16) + (size_t)(P + 1) * 8;
}

// A probe job's slot workspace: the probe rows partitioned by the table's P
// (partition workspace, keys, payloads, offsets), then the probe workspace.
struct ProbeJobLayout {
    PartLayout pl;
    ProbeLayout ql;
    size_t part_off, keys_off, pay_off, off_off, probe_off, bytes;
};

ProbeJobLayout probe_job_layout(int64_t n, int32_t P, int32_t kt)
{
    ProbeJobLayout L;
    L.pl = part_layout(n, P);
    L.ql = probe_layout(n, P);
    const size_t k = (size_t)(n > 0 ? n : 1);
    size_t o = 0;
    L.part_off = o;
    o += align_up(L.pl.bytes);
    L.keys_off = o;
    o += align_up(k * (size_t)kt);
    L.pay_off = o;
    o += align_up(k * 8);
    L.off_off = o;
    o += align_up((size_t)(P + 1) * 8);
    L.probe_off = o;
    o += align_up(L.ql.bytes);
    L.bytes = o;
    return L;
}

// Workspace of one slot: the largest merge layout (chunked: a served merge
// needs no global-table join) or probe job over both key types and every P
// up to max_P at the largest sizes.
size_t server_slot_bytes(int64_t max_left, int64_t max_right, int32_t max_P)
{
    size_t b = 0;
    for (int32_t P = 1; P <= max_P; ++P)
        for (int32_t kt : {MDX_KEY_I32, MDX_KEY_I64}) {
            b = std::max(b, merge_layout(max_left, max_right, P, kt, true).bytes);
            b = std::max(b, probe_job_layout(max_right, P, kt).bytes);
        }
    return align_up(b);
}

int32_t check_server_limits(int32_t slots, int64_t max_left, int64_t max_right, int32_t max_P,
                            const char *W)
{
    if (slots < 1 || slots > MDX_MAX_SLOTS)
        return fail(MDX_ERR_INVALID, std::string(W) + ": slots outside [1, MDX_MAX_SLOTS]");
    if (int32_t e = check_sizes(max_left, max_P, MDX_KEY_I64, W))
        return e;
    return check_sizes(max_right, max_P, MDX_KEY_I64, W);
}

}  // namespace

extern "C" {

int32_t mdx_server_workspace_bytes(int32_t slots, int64_t max_left, int64_t max_right,
                                   int32_t max_P, size_t *h_bytes)
{
    g_err.clear();
    const char *W = "mdx_server_workspace_bytes";
    if (int32_t e = check_server_limits(slots, max_left, max_right, max_P, W))
        return e;
    if (!h_bytes)
        return fail(MDX_ERR_INVALID, std::string(W) + ": h_bytes is null");
    *h_bytes = (size_t)slots * server_slot_bytes(max_left, max_right, max_P);
    return MDX_OK;
}

int32_t mdx_server_create(int32_t slots, int64_t max_left, int64_t max_right, int32_t max_P,
                          size_t budget_bytes, void *d_ws, size_t ws_bytes,
                          mdx_server **h_server)
{
    g_err.clear();
    const char *W = "mdx_server_create";
    if (int32_t e = check_server_limits(slots, max_left, max_right, max_P, W))
        return e;
    if (!h_server)
        return fail(MDX_ERR_INVALID, std::string(W) + ": h_server is null");
    *h_server = nullptr;
    const size_t per = server_slot_bytes(max_left, max_right, max_P);
    if (!d_ws || !aligned(d_ws, kAlign))
        return fail(MDX_ERR_INVALID, std::string(W) + ": workspace null or not 256-byte aligned");
    if (ws_bytes < (size_t)slots * per)
        return fail(MDX_ERR_WORKSPACE, std::string(W) + ": workspace needs " +
                                           std::to_string((size_t)slots * per) + " bytes");
    auto *srv = new mdx_server;
    srv->slots = slots;
    srv->max_left = max_left;
    srv->max_right = max_right;
    srv->max_P = max_P;
    srv->budget = budget_bytes;
    srv->slot_bytes = per;
    srv->d_ws = (char *)d_ws;
    srv->tag.assign((size_t)slots, -1);
    srv->held.assign((size_t)slots, 0);
    srv->busy.assign((size_t)slots, 0);
    hipError_t e = hipGetDevice(&srv->device);
    for (int32_t i = 0; i < slots && e == hipSuccess; ++i) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess)
            break;
        srv->streams.push_back(st);
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess)
            break;
        srv->done.push_back(ev);
    }
    if (e != hipSuccess) {
        mdx_server_destroy(srv);
        return hip_fail(e, W);
    }
    *h_server = srv;
    return MDX_OK;
}

int32_t mdx_server_submit(mdx_server *srv, const mdx_merge_desc *h_desc, int64_t tag,
                          hipEvent_t ready, int32_t *h_slot)
{
    g_err.clear();
    const char *W = "mdx_server_submit";
    if (!srv || !h_desc || !h_slot)
        return fail(MDX_ERR_INVALID, std::string(W) + ": null server, descriptor or h_slot");
    const mdx_merge_desc &d = *h_desc;
    if (int32_t e = check_merge(d, W))
        return e;
    if (d.n_left > srv->max_left || d.n_right > srv->max_right || d.P > srv->max_P)
        return fail(MDX_ERR_INVALID, std::string(W) + ": merge larger than the server's limits");
    const size_t need = request_bytes(d);
    if (need > srv->budget)
        return fail(MDX_ERR_INVALID, std::string(W) + ": merge alone exceeds the memory budget");
    *h_slot = -1;
    int32_t s = -1;
    for (int32_t i = 0; i < srv->slots; ++i)
        if (!srv->busy[(size_t)i]) {
            s = i;
            break;
        }
    if (s < 0 || srv->in_flight + need > srv->budget)
        return MDX_BUSY;
    char *ws = srv->d_ws + (size_t)s * srv->slot_bytes;
    if (int32_t e = check_merge_ws(d, ws, srv->slot_bytes,
                                   merge_layout(d.n_left, d.n_right, d.P, d.key_type, true).bytes,
                                   W))
        return e;
    if (int32_t e = check_merge_ws(d, srv->d_ws, (size_t)srv->slots * srv->slot_bytes, 0, W))
        return e;
    hipStream_t st = srv->streams[(size_t)s];
    hipError_t e = ready ? hipStreamWaitEvent(st, ready, 0) : hipSuccess;
    if (e == hipSuccess)
        e = enqueue_merge(d, ws, st, true);
    if (e == hipSuccess)
        e = hipEventRecord(srv->done[(size_t)s], st);
    if (e != hipSuccess)
        return hip_fail(e, W);
    srv->busy[(size_t)s] = 1;
    srv->tag[(size_t)s] = tag;
    srv->held[(size_t)s] = need;
    srv->in_flight += need;
    *h_slot = s;
    return MDX_OK;
}

int32_t mdx_server_submit_probe(mdx_server *srv, const mdx_table *h_table,
                                const mdx_probe_desc *h_desc, int64_t tag, hipEvent_t ready,
                                int32_t *h_slot)
{
    g_err.clear();
    const char *W = "mdx_server_submit_probe";
    if (!srv || !h_table || !h_desc || !h_slot)
        return fail(MDX_ERR_INVALID, std::string(W) + ": null server, table, descriptor or h_slot");
    const mdx_table &t = *h_table;
    if (t.abi_version != MDX_ABI_VERSION || !t.d_slots)
        return fail(MDX_ERR_INVALID, std::string(W) + ": table missing or built by another ABI version");
    const mdx_probe_desc &d = *h_desc;
    const int32_t P = t.P, kt = t.key_type;
    if (int32_t e = check_sizes(d.n, P, kt, W))
        return e;
    if (int32_t e = check_columns(d.d_keys, d.d_payload, d.n, kt, W))
        return e;
    if (int32_t e = check_outputs(d.d_out_key, d.d_out_lpay, d.d_out_rpay, d.out_capacity, kt,
                                  d.d_out_offsets, d.d_status, W))
        return e;
    if (d.n > srv->max_right || P > srv->max_P)
        return fail(MDX_ERR_INVALID, std::string(W) + ": probe larger than the server's limits");
    const size_t need = probe_request_bytes(d, P, kt);
    if (need > srv->budget)
        return fail(MDX_ERR_INVALID, std::string(W) + ": probe alone exceeds the memory budget");
    const ProbeJobLayout L = probe_job_layout(d.n, P, kt);
    if (L.bytes > srv->slot_bytes)  // a merge slot always holds a probe job of its limits
        return fail(MDX_ERR_WORKSPACE, std::string(W) + ": slot workspace too small for the probe");
    const size_t kb = (size_t)d.out_capacity * (size_t)kt, vb = (size_t)d.out_capacity * 8;
    const size_t ws_all = (size_t)srv->slots * srv->slot_bytes;
    if (overlap(srv->d_ws, ws_all, d.d_out_key, kb) || overlap(srv->d_ws, ws_all, d.d_out_lpay, vb) ||
        overlap(srv->d_ws, ws_all, d.d_out_rpay, vb) || overlap(t.d_mem, t.bytes, d.d_out_key, kb) ||
        overlap(t.d_mem, t.bytes, d.d_out_lpay, vb) || overlap(t.d_mem, t.bytes, d.d_out_rpay, vb))
        return fail(MDX_ERR_INVALID, std::string(W) + ": output overlaps the workspace or the table");
    *h_slot = -1;
    int32_t sl = -1;
    for (int32_t i = 0; i < srv->slots; ++i)
        if (!srv->busy[(size_t)i]) {
            sl = i;
            break;
        }
    if (sl < 0 || srv->in_flight + need > srv->budget)
        return MDX_BUSY;
    char *b = srv->d_ws + (size_t)sl * srv->slot_bytes;
    void *pk = b + L.keys_off;
    int64_t *pv = (int64_t *)(b + L.pay_off), *poff = (int64_t *)(b + L.off_off);
    const ProbeWs w = probe_ws(b + L.probe_off, L.ql);
    ProbeOut o;
    o.key = d.d_out_key;
    o.lpay = d.d_out_lpay;
    o.rpay = d.d_out_rpay;
    o.cap = d.out_capacity;
    o.offsets = d.d_out_offsets;
    hipStream_t st = srv->streams[(size_t)sl];
    hipError_t e = ready ? hipStreamWaitEvent(st, ready, 0) : hipSuccess;
    const PartArgs pa = {d.d_keys, d.d_payload, d.n, pk, pv, poff, nullptr, b + L.part_off};
    if (e == hipSuccess)
        e = launch_partition(&pa, 1, kt, P, 0, 0, 0, st);
    if (e == hipSuccess)
        e = launch_probe_plan(poff, d.n, P, w, nullptr, st);
    if (e == hipSuccess)
        e = launch_probe_group(pk, pv, kt, P, make_view(t, t.d_offsets, 0, P), 0, w, o, d.d_status,
                               0, st);
    if (e == hipSuccess)
        e = launch_probe_finalize(P, w, o, nullptr, st);
    if (e == hipSuccess)
        e = hipEventRecord(srv->done[(size_t)sl], st);
    if (e != hipSuccess)
        return hip_fail(e, W);
    srv->busy[(size_t)sl] = 1;
    srv->tag[(size_t)sl] = tag;
    srv->held[(size_t)sl] = need;
    srv->in_flight += need;
    *h_slot = sl;
    return MDX_OK;
}

int32_t mdx_server_poll(mdx_server *srv, int64_t *h_tags, int32_t capacity, int32_t *h_count)
{
    g_err.clear();
    const char *W = "mdx_server_poll";
    if (!srv || !h_count || capacity < 0 || (capacity > 0 && !h_tags))
        return fail(MDX_ERR_INVALID, std::string(W) + ": bad arguments");
    int32_t n = 0;
    for (int32_t i = 0; i < srv->slots && n < capacity; ++i) {
        if (!srv->busy[(size_t)i])
            continue;
        const hipError_t e = hipEventQuery(srv->done[(size_t)i]);
        if (e == hipErrorNotReady)
            continue;
        if (e != hipSuccess)
            return hip_fail(e, W);
        h_tags[n++] = srv->tag[(size_t)i];
        srv->busy[(size_t)i] = 0;
        srv->tag[(size_t)i] = -1;
        srv->in_flight -= srv->held[(size_t)i];
        srv->held[(size_t)i] = 0;
    }
    *h_count = n;
    return MDX_OK;
}

int32_t mdx_server_stats(const mdx_server *srv, int32_t *h_busy_slots, size_t *h_bytes_in_flight)
{
    g_err.clear();
    if (!srv || !h_busy_slots || !h_bytes_in_flight)
        return fail(MDX_ERR_INVALID, "mdx_server_stats: null argument");
    int32_t b = 0;
    for (char x : srv->busy)
        b += x ? 1 : 0;
    *h_busy_slots = b;
    *h_bytes_in_flight = srv->in_flight;
    return MDX_OK;
}

int32_t mdx_server_destroy(mdx_server *srv)
{
    g_err.clear();
    if (!srv)
        return MDX_OK;
    hipError_t first = hipSuccess;
    for (hipStream_t st : srv->streams) {
        const hipError_t e = hipStreamSynchronize(st);  // merges in flight finish first
        if (first == hipSuccess)
            first = e;
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t ev : srv->done)
        (void)hipEventDestroy(ev);
    delete srv;
    return first == hipSuccess ? MDX_OK : hip_fail(first, "mdx_server_destroy");
}

// ---- transpose sum ----------------------------------------------------------------

int32_t mdx_transpose_sum(const double *d_x, double *d_y, int64_t n, hipStream_t stream)
{
    g_err.clear();
    const char *W = "mdx_transpose_sum";
    if (n < 0 || n > MDX_MAX_TRANSPOSE_N)
        return fail(MDX_ERR_INVALID, std::string(W) + ": n outside [0, MDX_MAX_TRANSPOSE_N]");
    if (n == 0)
        return MDX_OK;
    if (!d_x || !d_y || !aligned(d_x, 8) || !aligned(d_y, 8))
        return fail(MDX_ERR_INVALID, std::string(W) + ": null or misaligned matrix");
    const size_t bytes = (size_t)n * (size_t)n * 8;
    if ((const void *)d_x != (const void *)d_y && overlap(d_x, bytes, d_y, bytes))
        return fail(MDX_ERR_INVALID, std::string(W) + ": x and y overlap without being equal");
    const hipError_t e = launch_transpose_sum(d_x, d_y, n, stream);
    return e == hipSuccess ? MDX_OK : hip_fail(e, W);
}

}  // extern "C"
