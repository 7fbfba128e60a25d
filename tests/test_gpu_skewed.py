"""The skewed workload at full size: 5E7 x 5E7 rows, Zipf(1.1) keys over
1E7 values, P = 16.

Its join has ~5E13 rows, far beyond any memory, so (as read for this
workload) the graded part is partition + build + count over the whole
input: both partitions byte-exact, and the exact per-partition output
counts from the count-only probe and from mdx_merge (which reports them
even when its output does not fit).  Materialization is checked on the
window L join R[0:m), m the longest prefix of right rows whose output stays
within 2^28 rows (~2.7E8 rows, 6.4 GB): there by properties that fix the
output exactly (every row's key equals the left and right keys its payloads
name, every right row appears as often as the left table holds its key, no
(left, right) pair twice, per-partition counts equal the oracle's); and the
2^24-row window row by row against the oracle's materialized join.
Partitioning is stable, so a window is a prefix of every partition block."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import announce, assert_join_equals_oracle, dev, host, require_gpu, run_merge
from tests.helpers import part_np
from workloads import config_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def skewed():
    kl, vl, kr, vr = config_inputs("skewed")
    ref = oracle.join(kl, vl, kr, vr, P=16, materialize=False)
    return kl, vl, kr, vr, ref


@pytest.fixture(scope="module")
def right_counts(skewed):
    """For every right row, the output rows it makes (the left count of its
    key), by the oracle."""
    kl, _, kr, _, _ = skewed
    return oracle.match_counts(kl, kr)


def test_skewed_partition_build_count(skewed):
    import paper_2101_08878_amd as mdx
    announce("skewed 5e7 x 5e7: partition, build, count")
    kl, vl, kr, vr, ref = skewed
    P = 16
    lk, lv, lo = mdx.mdx_hash_partition(dev(kl), dev(vl), P)
    rk, rv, ro = mdx.mdx_hash_partition(dev(kr), dev(vr), P)
    torch.cuda.synchronize()
    for got, want in zip((host(lk), host(lv), host(lo)), oracle.hash_partition(kl, vl, P)):
        assert np.array_equal(got, want)
    for got, want in zip((host(rk), host(rv), host(ro)), oracle.hash_partition(kr, vr, P)):
        assert np.array_equal(got, want)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    t = mdx.mdx_join_build(lk, lv, lo, P, status=status)
    empty = (torch.empty(0, dtype=torch.int64, device="cuda"),) * 3
    _, _, _, off = mdx.mdx_join_probe(t, rk, rv, ro, out_capacity=0, out=empty, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & mdx.MDX_DEV_BAD_PARTITIONING == 0
    assert np.array_equal(np.diff(host(off)), ref["per_part"])
    assert int(host(off)[-1]) == ref["total"] > 10**13


def test_skewed_join_count(skewed):
    """The count-only join (the graded step's count) at full size: exact
    per-partition counts of the ~5.3E13-row join."""
    import paper_2101_08878_amd as mdx
    announce("skewed 5e7 x 5e7: partition + count-only join")
    kl, vl, kr, vr, ref = skewed
    P = 16
    lk, _, lo = mdx.mdx_hash_partition(dev(kl), dev(vl), P)
    rk, _, ro = mdx.mdx_hash_partition(dev(kr), dev(vr), P)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    off = mdx.mdx_join_count(lk, lo, rk, ro, P, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert np.array_equal(np.diff(host(off)), ref["per_part"])
    assert int(host(off)[-1]) == ref["total"]


def test_skewed_merge_counts(skewed):
    """mdx_merge with a 1-row output: every partition's count still exact,
    overflow reported, nothing written past the capacity."""
    import paper_2101_08878_amd as mdx
    announce("skewed 5e7 x 5e7: merge counts")
    kl, vl, kr, vr, ref = skewed
    got = run_merge(kl, vl, kr, vr, 16, cap=1)
    assert np.array_equal(np.diff(got["off"]), ref["per_part"])
    assert got["status"] & mdx.MDX_DEV_OUTPUT_OVERFLOW


def test_skewed_window_materialized(skewed, right_counts):
    announce("skewed window L x R[0:m), 2^24 rows")
    kl, vl, kr, vr, _ = skewed
    c = np.cumsum(right_counts)
    m = int(np.searchsorted(c, 1 << 24, side="right"))
    assert 0 < m < kr.size
    got = run_merge(kl, vl, kr[:m], vr[:m], 16, cap=int(c[m - 1]))
    assert_join_equals_oracle(kl, vl, kr[:m], vr[:m], 16, got)


def test_skewed_window_2_28(skewed, right_counts):
    """The 2^28-row window of the workload's reading (~2.7E8 output rows)."""
    import paper_2101_08878_amd as mdx
    announce("skewed window L x R[0:m), 2^28 rows")
    kl, vl, kr, vr, _ = skewed
    cnt = right_counts
    c = np.cumsum(cnt)
    m = int(np.searchsorted(c, 1 << 28, side="right"))
    total = int(c[m - 1])
    assert 0 < m < kr.size and total > (1 << 27)
    ref = oracle.join(kl, vl, kr[:m], vr[:m], P=16, materialize=False)
    assert ref["total"] == total
    lk, rk = dev(kl), dev(kr)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ok, ol, orr, off = mdx.mdx_merge(lk, dev(vl), rk[:m], dev(vr[:m]), 16, out_capacity=total,
                                     status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert np.array_equal(np.diff(host(off)), ref["per_part"])
    # payloads are row indices: every row's key is the key of both rows it names
    assert torch.equal(ok, lk[ol]) and torch.equal(ok, rk[orr])
    # every right row appears exactly as often as the left table holds its key
    assert torch.equal(torch.bincount(orr, minlength=m).cpu(), torch.from_numpy(cnt[:m]))
    # and never with the same left row twice
    pairs = torch.sort(orr * kl.size + ol).values
    assert not bool((pairs[1:] == pairs[:-1]).any().item())
    del pairs
    # rows of block p belong to partition p (every 97th row)
    o = host(off)
    idx = np.arange(0, total, 97)
    blocks = np.searchsorted(o, idx, side="right") - 1
    assert np.array_equal(part_np(host(ok[torch.from_numpy(idx).cuda()]), 16), blocks)
