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

mdx = pytest.importorskip("paper_2101_08878_amd")
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
                 "MDX_DEV_SCAN_TIMEOUT", "MDX_MAX_P",
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
