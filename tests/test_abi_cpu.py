"""Host-side checks of libmdx that need no GPU.

The library loads, exports every function include/mdx.h declares, the
binding's constants equal the header's, size queries are consistent, and
argument validation returns the documented status before enqueuing anything.
No call here reaches a kernel launch: every call with device pointers fails
validation first (the pointers are fake).
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdx.h")


def _ensure_library():
    """Build libmdx.so (hipcc cross-compiles for gfx950 without a GPU) when
    it is not there yet, so these host checks never skip silently."""
    lib = os.path.join(ROOT, "paper_2101_08878_amd", "libmdx.so")
    if not os.path.exists(lib):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "_mdx_build", os.path.join(ROOT, "paper_2101_08878_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()


_ensure_library()
import paper_2101_08878_amd as mdx  # noqa: E402
from paper_2101_08878_amd import _lib as L  # noqa: E402

FAKE = 1 << 40  # a 256-aligned address nothing dereferences


def _header():
    with open(HEADER) as f:
        return f.read()


def test_exports_every_declared_function():
    decl = set(re.findall(r"^\s*(?:int32_t|const char \*)\s*\*?\s*(mdx_\w+)\s*\(", _header(), re.M))
    assert decl == set(mdx.ABI_FUNCTIONS)
    lib = ctypes.CDLL(mdx.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name


def test_constants_match_header():
    h = _header()
    for name in ["MDX_OK", "MDX_ERR_INVALID", "MDX_ERR_WORKSPACE", "MDX_ERR_HIP", "MDX_KEY_I32",
                 "MDX_KEY_I64", "MDX_DEV_OUTPUT_OVERFLOW", "MDX_DEV_BAD_PARTITIONING",
                 "MDX_DEV_SCAN_TIMEOUT", "MDX_MAX_P", "MDX_BUSY", "MDX_MAX_LANES", "MDX_MAX_SLOTS",
                 "MDX_ABI_VERSION"]:
        m = re.search(rf"#define\s+{name}\s+(\d+)", h)
        assert m, name
        want = int(m.group(1))
        if name == "MDX_ABI_VERSION":
            assert mdx.abi_version() == want
        else:
            assert getattr(L, name) == want, name


def test_table_struct_layout():
    # 4 int32, int64, pointer, size_t, 6 pointers on LP64
    assert ctypes.sizeof(L.mdx_table) == 16 + 8 + 8 + 8 + 6 * 8


def test_status_strings():
    assert mdx.status_string(mdx.MDX_OK) == "ok"
    assert "invalid" in mdx.status_string(mdx.MDX_ERR_INVALID)
    assert "workspace" in mdx.status_string(mdx.MDX_ERR_WORKSPACE)
    assert mdx.status_string(12345) == "unknown status"


def test_size_queries():
    for P in [1, 3, 32, 4096]:
        a = mdx.mdx_hash_partition_workspace_bytes(1000, P)
        b = mdx.mdx_hash_partition_workspace_bytes(10**6, P)
        assert 0 < a <= b and a % 256 == 0
        t = mdx.mdx_join_table_bytes(10**6, P)
        assert t >= 10**6 * (2 * 16 + 2 * 8 + 8)
        m = mdx.mdx_merge_workspace_bytes(10**6, 2 * 10**6, P)
        assert m > t + mdx.mdx_join_probe_workspace_bytes(2 * 10**6, P)
    assert mdx.mdx_hash_partition_workspace_bytes(0, 4) > 0


@pytest.mark.parametrize("args", [(-1, 4, 8), (10, 0, 8), (10, 4097, 8), (10, 4, 2), (1 << 35, 4, 8)])
def test_size_query_rejects_bad_sizes(args):
    out = ctypes.c_size_t(0)
    assert L._part_ws(*args, ctypes.byref(out)) == mdx.MDX_ERR_INVALID
    assert mdx.last_error() != ""


def _part(**kw):
    a = dict(keys=FAKE, pay=FAKE + (1 << 30), n=100, kt=8, P=4, ko=FAKE + (2 << 30),
             vo=FAKE + (3 << 30), off=FAKE + (4 << 30), ws=FAKE + (5 << 30), wsb=1 << 20, s=None)
    a.update(kw)
    return L._part(a["keys"], a["pay"], a["n"], a["kt"], a["P"], a["ko"], a["vo"], a["off"],
                   a["ws"], a["wsb"], a["s"])


def test_partition_validation():
    E = mdx.MDX_ERR_INVALID
    assert _part(P=0) == E
    assert _part(P=4097) == E
    assert _part(n=-5) == E
    assert _part(kt=3) == E
    assert _part(keys=None) == E
    assert _part(off=None) == E
    assert _part(ko=FAKE) == E                  # output aliases input
    assert _part(pay=FAKE + 4) == E             # misaligned payload
    assert _part(ws=FAKE + (5 << 30) + 64) == E  # workspace not 256-aligned
    assert _part(wsb=16) == mdx.MDX_ERR_WORKSPACE
    assert "bytes" in mdx.last_error()


def test_build_probe_merge_validation():
    t = L.mdx_table()
    st = L._build(FAKE, FAKE + (1 << 30), FAKE + (2 << 30), 100, 4, 8, FAKE + (3 << 30), 16,
                  ctypes.byref(t), None, None)
    assert st == mdx.MDX_ERR_WORKSPACE
    st = L._build(FAKE, FAKE + (1 << 30), None, 100, 4, 8, FAKE + (3 << 30), 1 << 30,
                  ctypes.byref(t), None, None)
    assert st == mdx.MDX_ERR_INVALID
    # a table that was never built
    st = L._probe(ctypes.byref(L.mdx_table()), FAKE, FAKE, FAKE, 10, FAKE, 1 << 20, FAKE, FAKE,
                  FAKE, 10, FAKE, None, None)
    assert st == mdx.MDX_ERR_INVALID
    # merge: bad P, negative capacity, overlapping outputs, small workspace
    args = [FAKE, FAKE + (1 << 30), 10, FAKE + (2 << 30), FAKE + (3 << 30), 10, 8, 4,
            FAKE + (4 << 30), 1 << 30, FAKE + (5 << 30), FAKE + (6 << 30), FAKE + (7 << 30), 10,
            FAKE + (8 << 30), None, None]
    bad = list(args); bad[7] = 0
    assert L._merge(*bad) == mdx.MDX_ERR_INVALID
    bad = list(args); bad[13] = -1
    assert L._merge(*bad) == mdx.MDX_ERR_INVALID
    bad = list(args); bad[11] = bad[10]
    assert L._merge(*bad) == mdx.MDX_ERR_INVALID
    bad = list(args); bad[9] = 1024
    assert L._merge(*bad) == mdx.MDX_ERR_WORKSPACE
    bad = list(args); bad[2] = -3
    assert L._merge(*bad) == mdx.MDX_ERR_INVALID


def test_merge_desc_struct_layout():
    # 6 pointers/int64, 2 int32, 6 pointers/int64 on LP64, in the header's order
    assert ctypes.sizeof(L.mdx_merge_desc) == 6 * 8 + 2 * 4 + 6 * 8
    names = re.findall(r"^\s+[\w\s\*]*?\b(\w+);", _header().split("typedef struct mdx_merge_desc")[1]
                       .split("} mdx_merge_desc;")[0], re.M)
    assert names == [f[0] for f in L.mdx_merge_desc._fields_]


def _desc(nl, nr, P=4, kt=8, base=FAKE, cap=None):
    d = L.mdx_merge_desc()
    d.d_left_keys, d.d_left_payload, d.n_left = base, base + (1 << 30), nl
    d.d_right_keys, d.d_right_payload, d.n_right = base + (2 << 30), base + (3 << 30), nr
    d.key_type, d.P = kt, P
    d.d_out_key, d.d_out_lpay, d.d_out_rpay = base + (4 << 30), base + (5 << 30), base + (6 << 30)
    d.out_capacity = nr if cap is None else cap
    d.d_out_offsets, d.d_status = base + (7 << 30), None
    return d


def _batch_bytes(descs, lanes):
    arr = (L.mdx_merge_desc * max(len(descs), 1))(*descs)
    out = ctypes.c_size_t(0)
    st = L._batch_ws(len(descs), arr, lanes, ctypes.byref(out))
    return st, out.value


def test_batch_workspace_plan():
    a, b, c = _desc(100_000, 100_000, 8), _desc(60_000, 60_000, 4, 4), _desc(50_000, 50_000, 32)
    # a merge of a batch needs less than mdx_merge (no global-table join)
    ws = [_batch_bytes([d], 1)[1] for d in (a, b, c)]
    full = [mdx.mdx_merge_workspace_bytes(d.n_left, d.n_right, d.P, d.key_type) for d in (a, b, c)]
    assert all(w % 256 == 0 and 0 < w < f for w, f in zip(ws, full))
    assert _batch_bytes([], 4) == (mdx.MDX_OK, 0)
    assert _batch_bytes([a, b, c], 1) == (mdx.MDX_OK, max(ws))
    # largest first, each to the lane with the fewest rows: a | b, c
    assert _batch_bytes([c, b, a], 2) == (mdx.MDX_OK, ws[0] + max(ws[1], ws[2]))
    assert _batch_bytes([a, b, c], 3) == (mdx.MDX_OK, sum(ws))
    assert _batch_bytes([a, b, c], 8) == (mdx.MDX_OK, sum(ws))  # at most one lane per merge
    for lanes in [0, mdx.MDX_MAX_LANES + 1]:
        assert _batch_bytes([a], lanes)[0] == mdx.MDX_ERR_INVALID
    assert _batch_bytes([_desc(10, 10, P=0)], 2)[0] == mdx.MDX_ERR_INVALID
    out = ctypes.c_size_t(0)
    assert L._batch_ws(-1, None, 2, ctypes.byref(out)) == mdx.MDX_ERR_INVALID


def test_batch_validation():
    ws = FAKE + (64 << 30)
    good = [_desc(1000, 1000, base=FAKE + (i << 33)) for i in range(3)]
    st, need = _batch_bytes(good, 2)
    assert st == mdx.MDX_OK

    def run(descs, lanes=2, w=ws, wb=need):
        arr = (L.mdx_merge_desc * len(descs))(*descs)
        return L._batch(len(descs), arr, lanes, w, wb, None)

    bad = list(good); bad[1] = _desc(1000, 1000, P=0, base=FAKE + (1 << 33))
    assert run(bad) == mdx.MDX_ERR_INVALID
    assert "merge 1" in mdx.last_error()
    bad = list(good); bad[2] = _desc(1000, 1000, cap=-1, base=FAKE + (2 << 33))
    assert run(bad) == mdx.MDX_ERR_INVALID
    assert "merge 2" in mdx.last_error()
    assert run(good, wb=need - 256) == mdx.MDX_ERR_WORKSPACE
    assert run(good, w=ws + 64) == mdx.MDX_ERR_INVALID      # workspace not 256-aligned
    assert run(good, lanes=0) == mdx.MDX_ERR_INVALID
    # an output inside the batch workspace
    bad = list(good); bad[0] = _desc(1000, 1000, base=FAKE); bad[0].d_out_rpay = ws + 512
    assert run(bad) == mdx.MDX_ERR_INVALID
    assert L._batch(-1, None, 2, ws, need, None) == mdx.MDX_ERR_INVALID
    assert L._batch(2, None, 2, ws, need, None) == mdx.MDX_ERR_INVALID


def _fused_bytes(descs, tunings=None):
    arr = (L.mdx_merge_desc * max(len(descs), 1))(*descs)
    tarr = None
    if tunings is not None:
        tarr = (L.mdx_batch_tuning * len(tunings))()
        for i, (f, o, r, z) in enumerate(tunings):
            tarr[i].fill, tarr[i].fanout, tarr[i].part_rows, tarr[i].reserved = f, o, r, z
    lo, hi = ctypes.c_size_t(0), ctypes.c_size_t(0)
    st = L._fb_ws(len(descs), arr, tarr, ctypes.byref(lo), ctypes.byref(hi))
    return st, lo.value, hi.value


def test_fused_batch_workspace():
    a, b, c = _desc(100_000, 100_000, 8), _desc(60_000, 9_000, 4, 4), _desc(0, 5_000, 32)
    st, lo0, hi0 = _fused_bytes([])
    assert st == mdx.MDX_OK and lo0 == hi0
    st, lo1, hi1 = _fused_bytes([a])
    assert st == mdx.MDX_OK and lo1 == hi1 and lo1 > lo0
    st, lo, hi = _fused_bytes([a, b, c])
    assert st == mdx.MDX_OK and lo % 256 == 0 and hi % 256 == 0
    assert lo < hi  # the least workspace holds the largest merge, one wave holds all
    # per-merge workspace grows with either side
    prev = 0
    for n in [0, 1, 1000, 10**4, 10**5, 10**6]:
        st, lo_n, _ = _fused_bytes([_desc(n, 1000)])
        assert st == mdx.MDX_OK and lo_n >= prev
        prev = lo_n
    # tuning: fuller sub-buckets never need more workspace
    st, lo_f, _ = _fused_bytes([a], [(0.9, 0, 0, 0)])
    st2, lo_e, _ = _fused_bytes([a], [(0.3, 0, 0, 0)])
    assert st == st2 == mdx.MDX_OK and lo_f <= lo_e


@pytest.mark.parametrize("tuning", [(0.01, 0, 0, 0), (1.5, 0, 0, 0), (float("nan"), 0, 0, 0),
                                    (0.8, -1, 0, 0), (0.8, mdx.MDX_MAX_P + 1, 0, 0),
                                    (0.8, 128, 4, 0), (0.8, 128, 8, 1)])
def test_fused_batch_rejects_bad_tuning(tuning):
    st, _, _ = _fused_bytes([_desc(1000, 1000), _desc(10, 10)], [(0, 0, 0, 0), tuning])
    assert st == mdx.MDX_ERR_INVALID
    assert "merge 1" in mdx.last_error()


def test_fused_batch_create_validation():
    """Every check mdx_batch_create makes before its pinned allocation."""
    good = [_desc(1000, 1000, base=FAKE + (i << 33)) for i in range(3)]
    st, lo, hi = _fused_bytes(good)
    assert st == mdx.MDX_OK
    ws = FAKE + (64 << 30)
    h = ctypes.c_void_p()

    def create(descs, w=ws, wb=hi, tun=None):
        arr = (L.mdx_merge_desc * max(len(descs), 1))(*descs)
        return L._fb_create(len(descs), arr, tun, w, wb, ctypes.byref(h))

    assert create(good, wb=lo - 256) == mdx.MDX_ERR_WORKSPACE
    assert create(good, w=ws + 64) == mdx.MDX_ERR_INVALID
    assert create(good, w=None) == mdx.MDX_ERR_INVALID
    bad = list(good); bad[1] = _desc(1000, 1000, P=0, base=FAKE + (1 << 33))
    assert create(bad) == mdx.MDX_ERR_INVALID and "merge 1" in mdx.last_error()
    bad = list(good); bad[2] = _desc(1000, 1000, cap=-1, base=FAKE + (2 << 33))
    assert create(bad) == mdx.MDX_ERR_INVALID and "merge 2" in mdx.last_error()
    bad = list(good); bad[0] = _desc(1000, 1000, base=FAKE); bad[0].d_out_key = ws + 4096
    assert create(bad) == mdx.MDX_ERR_INVALID  # an output inside the workspace
    assert L._fb_create(-1, None, None, ws, hi, ctypes.byref(h)) == mdx.MDX_ERR_INVALID
    assert L._fb_create(2, None, None, ws, hi, ctypes.byref(h)) == mdx.MDX_ERR_INVALID
    arr = (L.mdx_merge_desc * 3)(*good)
    assert L._fb_create(3, arr, None, ws, hi, None) == mdx.MDX_ERR_INVALID
    assert L._fb_run(None, None) == mdx.MDX_ERR_INVALID
    assert L._fb_destroy(None) == mdx.MDX_OK
    w, n = ctypes.c_int32(), ctypes.c_int32()
    assert L._fb_info(None, ctypes.byref(w), ctypes.byref(n)) == mdx.MDX_ERR_INVALID


def test_autotune_lookup_reads_cells(tmp_path):
    import json
    from paper_2101_08878_amd import autotune
    path = str(tmp_path / "t.json")
    cells = [{"key_bytes": 8, "lo": 1000, "hi": 4000, "tuning": {"fill": 0.5, "fanout": 32,
                                                                 "part_rows": 2}}]
    with open(path, "w") as f:
        json.dump({"cells": cells}, f)
    assert autotune.lookup(8, 1000, path) == {"fill": 0.5, "fanout": 32, "part_rows": 2}
    assert autotune.lookup(8, 3999, path)["fanout"] == 32
    assert autotune.lookup(8, 4000, path) == {}
    assert autotune.lookup(4, 2000, path) == {}
    assert autotune.lookup(8, 2000, str(tmp_path / "missing.json")) == {}


def test_join_count_validation():
    """mdx_join_count's sizing and every check before a launch."""
    need = mdx.mdx_join_count_workspace_bytes(10**6, 2 * 10**6, 16)
    assert need % 256 == 0 and need >= 16 * (2 * 10**6 + 16 * 16)
    assert mdx.mdx_join_count_workspace_bytes(10**6, 10**9, 16) == need  # build side sizes it
    out = ctypes.c_size_t(0)
    assert L._count_ws(-1, 10, 4, 8, ctypes.byref(out)) == mdx.MDX_ERR_INVALID
    assert L._count_ws(10, 10, 0, 8, ctypes.byref(out)) == mdx.MDX_ERR_INVALID
    assert L._count_ws(10, 10, 4, 2, ctypes.byref(out)) == mdx.MDX_ERR_INVALID
    need = mdx.mdx_join_count_workspace_bytes(1000, 2000, 4)
    ws, offs = FAKE + (64 << 30), FAKE + (70 << 30)

    def call(lk=FAKE, lo=FAKE + 4096, nl=1000, rk=FAKE + (1 << 30), ro=FAKE + 8192, nr=2000, P=4,
             kt=8, w=ws, wb=need, out=offs, st=None):
        return L._count(lk, lo, nl, rk, ro, nr, P, kt, w, wb, out, st, None)

    assert call(wb=need - 256) == mdx.MDX_ERR_WORKSPACE
    assert call(lk=None) == mdx.MDX_ERR_INVALID
    assert call(rk=FAKE + 4) == mdx.MDX_ERR_INVALID            # misaligned int64 keys
    assert call(lo=None) == mdx.MDX_ERR_INVALID
    assert call(ro=FAKE + 3) == mdx.MDX_ERR_INVALID
    assert call(out=None) == mdx.MDX_ERR_INVALID
    assert call(st=FAKE + 2) == mdx.MDX_ERR_INVALID
    assert call(w=ws + 64) == mdx.MDX_ERR_INVALID
    assert call(out=ws + 512) == mdx.MDX_ERR_INVALID           # output inside the workspace
    assert call(P=0) == mdx.MDX_ERR_INVALID
    assert call(kt=5) == mdx.MDX_ERR_INVALID


def test_merge_workspace_monotone_in_both_sides():
    """A server slot and a batch lane are sized at the largest merge they
    take, which covers every smaller one only if a merge's workspace never
    shrinks as either side grows (the sub-bucket split depends on the larger
    side)."""
    sizes = [0, 1, 500, 7_680, 7_681, 10**4, 5 * 10**4, 10**5, 3 * 10**5, 10**6, 4 * 10**6,
             2 * 10**7, 10**8]
    for P in (1, 3, 8, 32, 257):
        for kt in (4, 8):
            ws = [[mdx.mdx_merge_workspace_bytes(a, b, P, kt) for b in sizes] for a in sizes]
            for i in range(len(sizes)):
                for j in range(len(sizes)):
                    if i + 1 < len(sizes):
                        assert ws[i + 1][j] >= ws[i][j], (P, kt, sizes[i], sizes[j])
                    if j + 1 < len(sizes):
                        assert ws[i][j + 1] >= ws[i][j], (P, kt, sizes[i], sizes[j])


def test_server_workspace_and_validation():
    """Server sizing and every argument check that runs before a stream or
    event is created (no GPU needed)."""
    # a slot holds a served merge (no global-table join: less than mdx_merge
    # needs) of the limits, or a probe job of max_right rows
    per = mdx.mdx_server_workspace_bytes(1, 10**6, 2 * 10**6, 8)
    full = max(mdx.mdx_merge_workspace_bytes(10**6, 2 * 10**6, P, kt)
               for P in range(1, 9) for kt in (4, 8))
    lane = max(_batch_bytes([_desc(10**6, 2 * 10**6, P, kt)], 1)[1]
               for P in range(1, 9) for kt in (4, 8))
    assert per % 256 == 0 and lane <= per < full
    assert mdx.mdx_server_workspace_bytes(3, 10**6, 2 * 10**6, 8) == 3 * per
    probe_only = mdx.mdx_server_workspace_bytes(1, 0, 2 * 10**6, 8)
    assert probe_only >= mdx.mdx_join_probe_workspace_bytes(2 * 10**6, 8, 8)
    out = ctypes.c_size_t(0)
    for args in [(0, 10, 10, 8), (mdx.MDX_MAX_SLOTS + 1, 10, 10, 8), (2, -1, 10, 8), (2, 10, 10, 0)]:
        assert L._srv_ws(*args, ctypes.byref(out)) == mdx.MDX_ERR_INVALID
    h = ctypes.c_void_p()
    need = mdx.mdx_server_workspace_bytes(2, 1000, 1000, 4)
    assert L._srv_create(0, 1000, 1000, 4, 1 << 30, FAKE, need, ctypes.byref(h)) == mdx.MDX_ERR_INVALID
    assert L._srv_create(2, 1000, 1000, 4, 1 << 30, FAKE, need - 256, ctypes.byref(h)) == mdx.MDX_ERR_WORKSPACE
    assert L._srv_create(2, 1000, 1000, 4, 1 << 30, FAKE + 64, need, ctypes.byref(h)) == mdx.MDX_ERR_INVALID
    assert L._srv_create(2, 1000, 1000, 4, 1 << 30, None, need, ctypes.byref(h)) == mdx.MDX_ERR_INVALID
    assert L._srv_create(2, 1000, 1000, 4, 1 << 30, FAKE, need, None) == mdx.MDX_ERR_INVALID
    slot, n = ctypes.c_int32(0), ctypes.c_int32(0)
    d = _desc(100, 100)
    assert L._srv_submit(None, ctypes.byref(d), 1, None, ctypes.byref(slot)) == mdx.MDX_ERR_INVALID
    assert L._srv_poll(None, None, 0, ctypes.byref(n)) == mdx.MDX_ERR_INVALID
    assert L._srv_destroy(None) == mdx.MDX_OK
    assert "busy" in mdx.status_string(mdx.MDX_BUSY)


def test_transpose_sum_validation():
    E = mdx.MDX_ERR_INVALID
    n = 100
    assert L._tsum(FAKE, FAKE + (1 << 30), -1, None) == E
    assert L._tsum(FAKE, FAKE + (1 << 30), (1 << 17) + 1, None) == E
    assert L._tsum(None, FAKE, n, None) == E
    assert L._tsum(FAKE + 4, FAKE + (1 << 30), n, None) == E       # misaligned
    assert L._tsum(FAKE, FAKE + 8 * n, n, None) == E                # partial overlap
    assert L._tsum(None, None, 0, None) == mdx.MDX_OK               # n = 0: nothing to do
    m = re.search(r"#define\s+MDX_MAX_TRANSPOSE_N\s+\(INT64_C\(1\)\s*<<\s*(\d+)\)", _header())
    assert m and L.MDX_MAX_TRANSPOSE_N == 1 << int(m.group(1))


def test_noalloc_partition_rejects_sizes_beyond_its_scratch():
    """mdx_hash_partition_noalloc checks its workspace need against the
    library's scratch array on the host and enqueues nothing when it does
    not fit (n = 1E8 fits P = 85, not P = 86)."""
    h = _header()
    m = re.search(r"#define\s+MDX_NOALLOC_SCRATCH_BYTES\s+\((\d+)u\s*<<\s*(\d+)\)", h)
    assert m and int(m.group(1)) << int(m.group(2)) == L.MDX_NOALLOC_SCRATCH_BYTES
    n = 100_000_000
    k, v, ko, vo, off = (FAKE + i * (1 << 32) for i in range(5))
    for P in (86, 128, 4096):
        need = mdx.mdx_hash_partition_workspace_bytes(n, P)
        assert need > L.MDX_NOALLOC_SCRATCH_BYTES
        st = L._part_noalloc(k, v, n, mdx.MDX_KEY_I64, P, ko, vo, off, None)
        assert st == mdx.MDX_ERR_WORKSPACE
        assert "scratch" in mdx.last_error()
    assert mdx.mdx_hash_partition_workspace_bytes(n, 85) <= L.MDX_NOALLOC_SCRATCH_BYTES
    # the usual argument checks come first
    assert L._part_noalloc(None, v, n, mdx.MDX_KEY_I64, 32, ko, vo, off, None) == mdx.MDX_ERR_INVALID
    assert L._part_noalloc(k, v, n, mdx.MDX_KEY_I64, 0, ko, vo, off, None) == mdx.MDX_ERR_INVALID
    assert L._part_noalloc(k, v, n, mdx.MDX_KEY_I64, 32, k, vo, off, None) == mdx.MDX_ERR_INVALID
