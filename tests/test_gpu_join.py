"""Parity of the staged join (mdx_join_build + mdx_join_probe) with the
oracle's sort-merge join.  Output row order is free, so rows are compared
after sorting by (left payload, right payload, key); the per-partition
output offsets are compared exactly."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import (announce, assert_join_equals_oracle, dev, host, require_gpu,
                            run_staged_join)
from workloads import config_inputs, edge_tables, match_fraction_tables, uniform_tables, zipf_tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_join_plain_workload():
    announce("join plain workload P=4")
    kl, vl, kr, vr = config_inputs("plain")
    got = run_staged_join(kl, vl, kr, vr, 4)
    assert_join_equals_oracle(kl, vl, kr, vr, 4, got)


@pytest.mark.parametrize("P", [1, 3, 8, 32, 257])
def test_join_unique_build_keys(P):
    announce(f"join unique build P={P}")
    kl, vl, kr, vr = match_fraction_tables(60_000, 70_001, 0.3, seed=P)
    got = run_staged_join(kl, vl, kr, vr, P)
    assert_join_equals_oracle(kl, vl, kr, vr, P, got)


@pytest.mark.parametrize("dtype", [np.int64, np.int32])
def test_join_repeated_keys(dtype):
    announce(f"join repeated keys {np.dtype(dtype).name}")
    kl, vl, kr, vr = uniform_tables(9_000, 11_000, 2_000, seed=4, key_dtype=dtype)
    got = run_staged_join(kl, vl, kr, vr, 16, cap=200_000)
    assert_join_equals_oracle(kl, vl, kr, vr, 16, got)


def test_join_skewed_large_fanout():
    """Zipf keys: some right rows match thousands of left rows, so the output
    of one probe tile spans many expansion chunks."""
    announce("join zipf fan-out")
    kl, vl, kr, vr = zipf_tables(12_000, 12_000, 1.1, 3_000, seed=2)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    got = run_staged_join(kl, vl, kr, vr, 16, cap=total)
    assert_join_equals_oracle(kl, vl, kr, vr, 16, got)


@pytest.mark.parametrize("name", ["empty_left", "empty_right", "both_empty", "all_equal", "extremes",
                                  "int32_negative", "int32_extremes"])
def test_join_edge_tables(name):
    announce(f"join edge {name}")
    kl, vl, kr, vr, _ = edge_tables(name)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    for P in [1, 5, 32]:
        got = run_staged_join(kl, vl, kr, vr, P, cap=max(total, 1))
        assert_join_equals_oracle(kl, vl, kr, vr, P, got)


def test_join_capacity_overflow_reports_exact_offsets():
    announce("join capacity overflow")
    kl, vl, kr, vr = uniform_tables(5_000, 5_000, 500, seed=8)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    got = run_staged_join(kl, vl, kr, vr, 8, cap=total // 3)
    assert got["off"][-1] == total
    import paper_2101_08878_amd as mdx
    assert got["status"] & mdx.MDX_DEV_OUTPUT_OVERFLOW
    assert_join_equals_oracle(kl, vl, kr, vr, 8, got)


def test_join_count_only():
    announce("join count only")
    import paper_2101_08878_amd as mdx
    kl, vl, kr, vr = uniform_tables(5_000, 6_000, 900, seed=9)
    P = 8
    lk, lv, lo = mdx.mdx_hash_partition(dev(kl), dev(vl), P)
    rk, rv, ro = mdx.mdx_hash_partition(dev(kr), dev(vr), P)
    t = mdx.mdx_join_build(lk, lv, lo, P)
    empty = (torch.empty(0, dtype=torch.int64, device="cuda"),) * 3
    _, _, _, off = mdx.mdx_join_probe(t, rk, rv, ro, out_capacity=0, out=empty)
    torch.cuda.synchronize()
    ref = oracle.join(kl, vl, kr, vr, P=P, materialize=False)
    assert np.array_equal(np.diff(host(off)), ref["per_part"])


def test_join_bad_partitioning_is_reported():
    """Unpartitioned input with offsets that claim a partitioning: rows whose
    destination disagrees are skipped and flagged; nothing faults."""
    announce("join bad partitioning")
    import paper_2101_08878_amd as mdx
    kl, vl, kr, vr = uniform_tables(4_000, 4_000, 1_000, seed=3)
    P = 4
    off = torch.tensor([0, 1000, 2000, 3000, 4000], dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    t = mdx.mdx_join_build(dev(kl), dev(vl), off, P, status=status)
    _, _, _, out_off = mdx.mdx_join_probe(t, dev(kr), dev(vr), off, out_capacity=4_000_000,
                                          status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & mdx.MDX_DEV_BAD_PARTITIONING
    assert host(out_off)[-1] <= oracle.join(kl, vl, kr, vr, materialize=False)["total"]


def test_table_reuse_across_probes():
    """One build, two probes of different right tables."""
    announce("join table reuse")
    import paper_2101_08878_amd as mdx
    kl, vl, kr, vr = uniform_tables(8_000, 8_000, 3_000, seed=11)
    _, _, kr2, vr2 = uniform_tables(8_000, 5_000, 3_000, seed=12)
    P = 8
    lk, lv, lo = mdx.mdx_hash_partition(dev(kl), dev(vl), P)
    t = mdx.mdx_join_build(lk, lv, lo, P)
    for k, v in [(kr, vr), (kr2, vr2)]:
        rk, rv, ro = mdx.mdx_hash_partition(dev(k), dev(v), P)
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        ok, ol, orr, off = mdx.mdx_join_probe(t, rk, rv, ro, out_capacity=100_000, status=status)
        torch.cuda.synchronize()
        got = dict(key=host(ok), lpay=host(ol), rpay=host(orr), off=host(off),
                   status=int(status.item()), cap=100_000)
        assert_join_equals_oracle(kl, vl, k, v, P, got)


# ---- count-only join (mdx_join_count) ----------------------------------------------------

def _count(kl, kr, P, lofs=None, rofs=None, status=None):
    import paper_2101_08878_amd as mdx
    pay_l = np.arange(kl.size, dtype=np.int64)
    pay_r = np.arange(kr.size, dtype=np.int64)
    if lofs is None:
        lk, _, lo = mdx.mdx_hash_partition(dev(kl), dev(pay_l), P)
        rk, _, ro = mdx.mdx_hash_partition(dev(kr), dev(pay_r), P)
    else:
        lk, lo, rk, ro = dev(kl), lofs, dev(kr), rofs
    off = mdx.mdx_join_count(lk, lo, rk, ro, P, status=status)
    torch.cuda.synchronize()
    return host(off)


@pytest.mark.parametrize("case", ["plain", "zipf", "all_equal", "unique", "int32_negative",
                                  "empty_left", "empty_right", "both_empty"])
@pytest.mark.parametrize("P", [1, 7, 64])
def test_join_count_matches_oracle(case, P):
    """Per-partition counts equal the oracle's: repeated keys on both sides
    (Zipf; one key 20000 times), distinct keys, negative int32 keys, empty
    sides, P = 1, 7 (not a power of two) and 64."""
    announce(f"join count {case} P={P}")
    from workloads import zipf_tables
    if case == "plain":
        kl, _, kr, _ = uniform_tables(40_000, 50_000, 30_000, seed=21)
    elif case == "zipf":
        kl, _, kr, _ = zipf_tables(60_000, 60_000, 1.1, 10_000, seed=22)
    elif case == "all_equal":
        kl, kr = np.full(20_000, 5, np.int64), np.concatenate([np.full(300, 5, np.int64),
                                                              np.arange(6, 4000, dtype=np.int64)])
    elif case == "unique":
        kl, _, kr, _ = match_fraction_tables(70_000, 90_000, 0.3, seed=23)
    else:
        kl, _, kr, _, _ = edge_tables(case)
    ref = oracle.join(kl, np.arange(kl.size, dtype=np.int64), kr, np.arange(kr.size, dtype=np.int64),
                      P=P, materialize=False)
    off = _count(kl, kr, P)
    assert off[0] == 0 and off[-1] == ref["total"]
    assert np.array_equal(np.diff(off), ref["per_part"])


def test_join_count_many_partitions_and_large_counts():
    """P = 4096, and one key with 3E5 copies on each side (9E10 output rows,
    beyond 32 bits)."""
    announce("join count P=4096 and a 9e10-row key")
    kl, _, kr, _ = uniform_tables(200_000, 200_000, 150_000, seed=24)
    ref = oracle.join(kl, np.arange(kl.size, dtype=np.int64), kr, np.arange(kr.size, dtype=np.int64),
                      P=4096, materialize=False)
    assert np.array_equal(np.diff(_count(kl, kr, 4096)), ref["per_part"])
    kl = np.concatenate([np.full(300_000, -7, np.int64), np.arange(1000, dtype=np.int64)])
    kr = np.concatenate([np.arange(500, 1500, dtype=np.int64), np.full(300_000, -7, np.int64)])
    off = _count(kl, kr, 3)
    ref = oracle.join(kl, np.arange(kl.size, dtype=np.int64), kr, np.arange(kr.size, dtype=np.int64),
                      P=3, materialize=False)
    assert np.array_equal(np.diff(off), ref["per_part"]) and off[-1] == 9 * 10**10 + 500


def test_join_count_bad_partitioning_is_reported():
    """Unpartitioned rows with offsets that claim a partitioning: flagged,
    skipped, nothing faults."""
    import paper_2101_08878_amd as mdx
    announce("join count bad partitioning")
    kl, _, kr, _ = uniform_tables(4_000, 4_000, 1_000, seed=3)
    P = 4
    off = torch.tensor([0, 1000, 2000, 3000, 4000], dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    got = _count(kl, kr, P, off, off, status)
    assert int(status.item()) & mdx.MDX_DEV_BAD_PARTITIONING
    assert got[-1] <= oracle.join(kl, np.zeros(kl.size, np.int64), kr, np.zeros(kr.size, np.int64),
                                  materialize=False)["total"]
