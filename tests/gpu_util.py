"""Helpers for the GPU parity tests (device transfer, running the C-ABI
calls through the binding, comparing with the oracle)."""

from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from tests.helpers import canonical, part_np


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def announce(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def run_partition(keys, pay, P):
    import paper_2101_08878_amd as mdx
    ko, vo, off = mdx.mdx_hash_partition(dev(keys), dev(pay), P)
    torch.cuda.synchronize()
    return host(ko), host(vo), host(off)


def run_staged_join(kl, vl, kr, vr, P, cap=None):
    """Partition both sides, build on the left, probe with the right."""
    import paper_2101_08878_amd as mdx
    lk, lv, lo = mdx.mdx_hash_partition(dev(kl), dev(vl), P)
    rk, rv, ro = mdx.mdx_hash_partition(dev(kr), dev(vr), P)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    t = mdx.mdx_join_build(lk, lv, lo, P, status=status)
    cap = max(len(kr), 1) if cap is None else cap
    ok, ol, orr, off = mdx.mdx_join_probe(t, rk, rv, ro, out_capacity=cap, status=status)
    torch.cuda.synchronize()
    return dict(key=host(ok), lpay=host(ol), rpay=host(orr), off=host(off),
                status=int(status.item()), cap=cap)


def run_merge(kl, vl, kr, vr, P, cap=None):
    import paper_2101_08878_amd as mdx
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    cap = max(len(kr), 1) if cap is None else cap
    ok, ol, orr, off = mdx.mdx_merge(dev(kl), dev(vl), dev(kr), dev(vr), P, out_capacity=cap,
                                     status=status)
    torch.cuda.synchronize()
    return dict(key=host(ok), lpay=host(ol), rpay=host(orr), off=host(off),
                status=int(status.item()), cap=cap)


def assert_join_equals_oracle(kl, vl, kr, vr, P, got):
    """Bit-exact after canonical ordering; per-partition blocks exact."""
    import paper_2101_08878_amd as mdx
    ref = oracle.join(kl, vl, kr, vr, P=P)
    total = ref["total"]
    off = got["off"]
    assert off[0] == 0 and off[-1] == total, (off[-1], total)
    assert np.array_equal(np.diff(off), ref["per_part"])
    assert got["status"] & mdx.MDX_DEV_BAD_PARTITIONING == 0
    if total > got["cap"]:
        assert got["status"] & mdx.MDX_DEV_OUTPUT_OVERFLOW
        return
    assert got["status"] == 0
    k = got["key"][:total].astype(np.int64)
    lp, rp = got["lpay"][:total], got["rpay"][:total]
    # every row of block p belongs to partition p
    dest = np.repeat(np.arange(P), np.diff(off))
    assert np.array_equal(part_np(k, P), dest)
    ck, cl, cr = canonical(k, lp, rp)
    assert np.array_equal(ck, ref["key"])
    assert np.array_equal(cl, ref["lpay"])
    assert np.array_equal(cr, ref["rpay"])
