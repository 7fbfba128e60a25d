"""mdx_hash_partition_noalloc (the partition with the library's own scratch
array instead of a caller workspace) against mdx_hash_partition: byte for
byte on two calls in a row, the second smaller than the first, and both
against the oracle's stable counting sort."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _with_workspace(keys, pay, P):
    import paper_2101_08878_amd as mdx
    ko, vo, off = mdx.mdx_hash_partition(keys, pay, P)
    torch.cuda.synchronize()
    return host(ko), host(vo), host(off)


def _without(keys, pay, P):
    import paper_2101_08878_amd as mdx
    n = keys.numel()
    # outputs start as garbage: every element must be written by the call
    ko = torch.full((n,), -5, dtype=keys.dtype, device=keys.device)
    vo = torch.full((n,), -7, dtype=torch.int64, device=keys.device)
    off = torch.full((P + 1,), -9, dtype=torch.int64, device=keys.device)
    mdx.mdx_hash_partition_noalloc(keys, pay, P, keys_out=ko, payload_out=vo, offsets=off)
    torch.cuda.synchronize()
    return host(ko), host(vo), host(off)


# (rows, P, key dtype) of consecutive calls; each later call is smaller, so
# stale counts of the earlier one sit in the scratch array past its end
CALLS = [
    [(1_000_003, 32, np.int64), (50_001, 7, np.int64)],
    [(3 * 4096 + 123, 4096, np.int32), (4097, 300, np.int32), (0, 5, np.int32)],
]


@pytest.mark.parametrize("calls", CALLS, ids=["int64", "int32"])
def test_noalloc_matches_workspace_call(calls):
    for i, (n, P, dt) in enumerate(calls):
        announce(f"noalloc call {i}: n={n} P={P} {np.dtype(dt).name}")
        rng = np.random.default_rng(1000 + i)
        info = np.iinfo(dt)
        k = rng.integers(info.min, info.max, n, dtype=np.int64, endpoint=True).astype(dt)
        v = np.arange(n, dtype=np.int64) * 5 + 3
        kd, vd = dev(k), dev(v)
        got = _without(kd, vd, P)
        ref = _with_workspace(kd, vd, P)
        want = oracle.hash_partition(k, v, P)
        for g, r, w in zip(got, ref, want):
            assert g.dtype == r.dtype
            assert np.array_equal(g, r)
            assert np.array_equal(g, w)


def test_noalloc_benchmark_sized_table():
    """1E8 rows at P = 32 (the benchmark's partition) fits the scratch
    array; the result equals the workspace call's."""
    announce("noalloc n=1E8 P=32")
    n = 100_000_000
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    k = torch.randperm(n, generator=g, device="cuda", dtype=torch.int64)
    v = torch.arange(n, dtype=torch.int64, device="cuda")
    import paper_2101_08878_amd as mdx
    ko, vo, off = mdx.mdx_hash_partition(k, v, 32)
    ko2 = torch.empty_like(k)
    vo2 = torch.empty_like(v)
    off2 = torch.empty(33, dtype=torch.int64, device="cuda")
    mdx.mdx_hash_partition_noalloc(k, v, 32, keys_out=ko2, payload_out=vo2, offsets=off2)
    torch.cuda.synchronize()
    assert torch.equal(off, off2)
    assert torch.equal(ko, ko2)
    assert torch.equal(vo, vo2)
