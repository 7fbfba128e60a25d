"""Parity of mdx_merge with the oracle.

mdx_merge partitions both tables, splits every partition into LDS-sized
sub-buckets and joins each sub-bucket in LDS; when a build sub-bucket is too
large for LDS (heavily repeated keys) the device switches to the global-table
join.  Both routes are compared with the oracle here, plus the 1E8 x 1E8
workload in the launch configuration the benchmark times, checked through
properties that hold at any size."""

import numpy as np
import pytest

import oracle
from tests.gpu_util import announce, assert_join_equals_oracle, require_gpu, run_merge
from tests.helpers import part_np
from workloads import config_inputs, edge_tables, match_fraction_tables, uniform_tables, zipf_tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_merge_plain_workload():
    announce("merge plain")
    kl, vl, kr, vr = config_inputs("plain")
    got = run_merge(kl, vl, kr, vr, 4)
    assert_join_equals_oracle(kl, vl, kr, vr, 4, got)


@pytest.mark.parametrize("scale", [0.02, 0.05])
def test_merge_paper_shape_reduced(scale):
    """The 1E8 workload's generator at 2E6 and 5E6 rows per side, P = 32
    (both split passes active)."""
    announce(f"merge paper x{scale}")
    kl, vl, kr, vr = config_inputs("paper", scale=scale)
    got = run_merge(kl, vl, kr, vr, 32)
    assert_join_equals_oracle(kl, vl, kr, vr, 32, got)


@pytest.mark.parametrize("P", [1, 3, 7, 64, 257, 4096])
def test_merge_partition_counts(P):
    announce(f"merge P={P}")
    kl, vl, kr, vr = match_fraction_tables(400_000, 300_001, 0.3, seed=P)
    got = run_merge(kl, vl, kr, vr, P)
    assert_join_equals_oracle(kl, vl, kr, vr, P, got)


@pytest.mark.parametrize("dtype", [np.int64, np.int32])
def test_merge_repeated_keys_radix(dtype):
    """Repeated keys whose sub-buckets still fit LDS: chains hold equal keys."""
    announce(f"merge repeated keys {np.dtype(dtype).name}")
    kl, vl, kr, vr = uniform_tables(200_000, 150_000, 60_000, seed=6, key_dtype=dtype)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    got = run_merge(kl, vl, kr, vr, 8, cap=total)
    assert_join_equals_oracle(kl, vl, kr, vr, 8, got)


@pytest.mark.parametrize("nl,nr,frac,P,dtype", [
    (3_000, 200_000, 0.5, 2, np.int64),   # small build side, large probe side
    (6_000, 8_000, 1.0, 1, np.int64),     # one sub-bucket, every probe row matches
    (6_000, 8_000, 1.0, 1, np.int32),
    (6_000, 6_400, 1.0, 1, np.int64),
])
def test_merge_join_routes(nl, nr, frac, P, dtype):
    """Uneven sides and sub-buckets where every probe row matches, against
    the oracle."""
    announce(f"merge routes {nl}x{nr} f={frac} P={P} {np.dtype(dtype).name}")
    kl, vl, kr, vr = match_fraction_tables(nl, nr, frac, seed=nl + nr, key_dtype=dtype)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    got = run_merge(kl, vl, kr, vr, P, cap=total)
    assert got["status"] == 0
    assert_join_equals_oracle(kl, vl, kr, vr, P, got)


def test_merge_probe_sub_bucket_spans_batches():
    """One probe key repeated 20000 times: its sub-bucket holds more probe
    rows than one 8192-row batch, so the join counts and then writes it
    batch by batch (sub-buckets are sized by the larger side, so only a
    repeated probe key gets there)."""
    announce("merge probe key x 20000")
    rng = np.random.default_rng(21)
    kl = rng.permutation(50_000).astype(np.int64)
    kr = np.concatenate([np.full(20_000, 777, np.int64), rng.integers(0, 100_000, 30_000)])
    kr = kr[rng.permutation(kr.size)]
    vl, vr = np.arange(kl.size, dtype=np.int64), np.arange(kr.size, dtype=np.int64)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    for P in (1, 4):
        got = run_merge(kl, vl, kr, vr, P, cap=total)
        assert got["status"] == 0
        assert_join_equals_oracle(kl, vl, kr, vr, P, got)


def test_merge_some_sub_buckets_repeat_keys():
    """20 build keys appear twice among 300000 distinct ones: only the
    sub-buckets holding them have probe rows with two matches."""
    announce("merge mixed routes")
    rng = np.random.default_rng(12)
    base = rng.permutation(300_000).astype(np.int64)
    kl = np.concatenate([base, base[rng.integers(0, base.size, 20)]])
    kl = kl[rng.permutation(kl.size)]
    kr = np.concatenate([base[rng.integers(0, base.size, 90_000)],
                         rng.integers(300_000, 600_000, 210_000)])
    kr = kr[rng.permutation(kr.size)]
    vl, vr = np.arange(kl.size, dtype=np.int64), np.arange(kr.size, dtype=np.int64)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    got = run_merge(kl, vl, kr, vr, 8, cap=total)
    assert got["status"] == 0
    assert_join_equals_oracle(kl, vl, kr, vr, 8, got)


def test_merge_int32_keys():
    announce("merge int32")
    kl, vl, kr, vr = match_fraction_tables(300_000, 250_000, 0.3, seed=4, key_dtype=np.int32)
    got = run_merge(kl, vl, kr, vr, 8)
    assert_join_equals_oracle(kl, vl, kr, vr, 8, got)


def test_merge_fallback_for_oversized_sub_bucket():
    """20000 build rows of one key: one sub-bucket exceeds the LDS table, so
    the device must take the global-table join."""
    announce("merge fallback (one key x 20000)")
    rng = np.random.default_rng(1)
    kl = np.concatenate([np.full(20_000, 5, np.int64), rng.integers(10, 10_000, 30_000)])
    kr = np.concatenate([np.full(50, 5, np.int64), rng.integers(10, 10_000, 20_000)])
    kl, kr = kl[rng.permutation(kl.size)], kr[rng.permutation(kr.size)]
    vl, vr = np.arange(kl.size, dtype=np.int64), np.arange(kr.size, dtype=np.int64)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    got = run_merge(kl, vl, kr, vr, 4, cap=total)
    assert_join_equals_oracle(kl, vl, kr, vr, 4, got)


@pytest.mark.parametrize("b", [3455, 3456, 3457, 3840, 3841])
@pytest.mark.parametrize("P", [1, 4])
def test_merge_one_key_at_table_size(b, P):
    """A build side of one key repeated b times, so one sub-bucket of b rows:
    at most 3456 (a merge's LDS table, and then the build side fits one
    table, so the global-table kernels are not even launched) it is joined
    in LDS, beyond it the device takes the global-table join.  The probe
    side has 3 matching rows and 500 misses."""
    announce(f"merge one key x {b}, P={P}")
    rng = np.random.default_rng(b + P)
    kl = np.full(b, 7, np.int64)
    kr = np.concatenate([np.full(3, 7, np.int64), rng.integers(100, 300, 500)])
    kr = kr[rng.permutation(kr.size)]
    vl, vr = np.arange(kl.size, dtype=np.int64), np.arange(kr.size, dtype=np.int64)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    got = run_merge(kl, vl, kr, vr, P, cap=total)
    assert_join_equals_oracle(kl, vl, kr, vr, P, got)


def test_merge_skewed_reduced():
    announce("merge zipf reduced")
    kl, vl, kr, vr = zipf_tables(15_000, 15_000, 1.1, 10_000, seed=0)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    got = run_merge(kl, vl, kr, vr, 16, cap=total)
    assert_join_equals_oracle(kl, vl, kr, vr, 16, got)


@pytest.mark.parametrize("name", ["empty_left", "empty_right", "both_empty", "all_equal", "extremes",
                                  "int32_negative", "int32_extremes"])
def test_merge_edge_tables(name):
    announce(f"merge edge {name}")
    kl, vl, kr, vr, _ = edge_tables(name)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    for P in [1, 5, 32]:
        got = run_merge(kl, vl, kr, vr, P, cap=max(total, 1))
        assert_join_equals_oracle(kl, vl, kr, vr, P, got)


def test_merge_capacity_overflow():
    announce("merge capacity overflow")
    import paper_2101_08878_amd as mdx
    kl, vl, kr, vr = match_fraction_tables(100_000, 100_000, 0.5, seed=2)
    got = run_merge(kl, vl, kr, vr, 8, cap=10_000)
    assert got["off"][-1] == 50_000
    assert got["status"] & mdx.MDX_DEV_OUTPUT_OVERFLOW


def assert_paper_merge(kl, kr, P, got):
    """Left keys are a permutation of [0, n), so a right row matches iff its
    key is below n, and then exactly once: the output must be exactly the
    right rows with key < n, each paired with the unique left row holding
    its key (payload = row index), and partition p's block must hold exactly
    the output keys with destination p.  This fixes the output up to the
    order of rows inside a partition."""
    n = kl.size
    assert got["status"] == 0
    off = got["off"]
    total = int(off[-1])
    key, lp, rp = got["key"][:total], got["lpay"][:total], got["rpay"][:total]
    # every output row is a genuine match
    assert np.array_equal(kl[lp], key)
    assert np.array_equal(kr[rp], key)
    # completeness and no duplicates: the right payloads are exactly the hits
    hits = np.flatnonzero(kr < n)
    assert hits.size == total
    assert np.array_equal(np.sort(rp), hits)
    # partition blocks
    dest = np.repeat(np.arange(P), np.diff(off))
    assert np.array_equal(part_np(key, P), dest)
    return total


@pytest.mark.parametrize("P", [1, 2, 3])
def test_merge_placement_by_partition(P):
    """1.3E7 x 1.3E7 (the 1E8 workload's generator): at P = 1 and 2 a
    partition holds 8192 or 4096 sub-buckets, at least 8 per workgroup of the
    join, so its output rows are placed by partition cursor and a chained scan
    over partitions; at P = 3 (2048) by the chained scan over sub-buckets."""
    announce(f"merge placement P={P}")
    kl, vl, kr, vr = config_inputs("paper", scale=0.13)
    got = run_merge(kl, vl, kr, vr, P)
    assert assert_paper_merge(kl, kr, P, got) == round(0.3 * kl.size)


@pytest.mark.parametrize("P", [32, 1])
def test_merge_paper_scale_properties(P):
    """1E8 x 1E8, P = 32 (what the benchmark times) and P = 1 (its secondary
    figure, output placed by partition cursor): |J| = 3E7, checked row by
    row as in assert_paper_merge."""
    announce(f"merge paper scale 1e8 P={P}")
    n = 100_000_000
    kl, vl, kr, vr = config_inputs("paper")
    got = run_merge(kl, vl, kr, vr, P, cap=n)
    assert assert_paper_merge(kl, kr, P, got) == 30_000_000
