"""Pins of the CPU oracle against things other than itself.

* fmix64: the published SMHasher verification value of MurmurHash3_x64_128
  (fmix64 is its finalizer), fmix64(0) = 0, and bijectivity via an inverse
  derived from the mathematics (xor-shift by >= 32 bits is an involution,
  odd multipliers are units mod 2^64).
* destination: unsigned remainder semantics, int32 sign extension.
* partition: numpy's stable argsort of the destinations (a library routine),
  and the stable-partition invariants.
* join: nested-loop brute force, pandas.merge (a library routine), a
  hand-worked example, closed-form cardinalities.
"""

import os

import numpy as np
import pandas as pd
import pytest

import oracle
from tests.helpers import (
    M64,
    brute_force_join,
    canonical,
    check_join_rows,
    check_partition_invariants,
    expected_cardinality,
    fmix64_np,
    part_np,
)
from workloads import config_inputs, edge_tables, match_fraction_tables, uniform_tables, zipf_tables


# --------------------------------------------------------------------------
# fmix64
# --------------------------------------------------------------------------

def _rotl(x, r):
    return ((x << r) | (x >> (64 - r))) & M64


def murmur3_x64_128(data: bytes, seed: int, fmix) -> bytes:
    """MurmurHash3_x64_128 (Appleby), body written from its published
    definition; ``fmix`` is the finalizer under test."""
    c1, c2 = 0x87C37B91114253D5, 0x4CF5AD432745937F
    n = len(data)
    h1 = h2 = seed & M64
    nblocks = n // 16
    for i in range(nblocks):
        k1 = int.from_bytes(data[16 * i:16 * i + 8], "little")
        k2 = int.from_bytes(data[16 * i + 8:16 * i + 16], "little")
        k1 = (k1 * c1) & M64
        k1 = _rotl(k1, 31)
        k1 = (k1 * c2) & M64
        h1 ^= k1
        h1 = _rotl(h1, 27)
        h1 = (h1 + h2) & M64
        h1 = (h1 * 5 + 0x52DCE729) & M64
        k2 = (k2 * c2) & M64
        k2 = _rotl(k2, 33)
        k2 = (k2 * c1) & M64
        h2 ^= k2
        h2 = _rotl(h2, 31)
        h2 = (h2 + h1) & M64
        h2 = (h2 * 5 + 0x38495AB5) & M64
    tail = data[16 * nblocks:]
    if len(tail) > 8:
        k2 = int.from_bytes(tail[8:], "little")
        k2 = (k2 * c2) & M64
        k2 = _rotl(k2, 33)
        k2 = (k2 * c1) & M64
        h2 ^= k2
    if len(tail) > 0:
        k1 = int.from_bytes(tail[:8], "little")
        k1 = (k1 * c1) & M64
        k1 = _rotl(k1, 31)
        k1 = (k1 * c2) & M64
        h1 ^= k1
    h1 ^= n
    h2 ^= n
    h1 = (h1 + h2) & M64
    h2 = (h2 + h1) & M64
    h1 = fmix(h1)
    h2 = fmix(h2)
    h1 = (h1 + h2) & M64
    h2 = (h2 + h1) & M64
    return h1.to_bytes(8, "little") + h2.to_bytes(8, "little")


def _smhasher_verification(fmix) -> int:
    key = bytes(range(256))
    digests = b"".join(murmur3_x64_128(key[:i], 256 - i, fmix) for i in range(256))
    final = murmur3_x64_128(digests, 0, fmix)
    return int.from_bytes(final[:4], "little")


def _golden_int(path):
    with open(path) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    return int(lines[0], 16)


def test_fmix64_smhasher_verification(golden_dir):
    want = _golden_int(os.path.join(golden_dir, "murmur3_x64_128_verification.txt"))
    assert _smhasher_verification(oracle.fmix64) == want


def test_test_side_fmix64_matches_published_value(golden_dir):
    # tests.helpers.fmix64_np checks destinations at scale; pin it the same way
    want = _golden_int(os.path.join(golden_dir, "murmur3_x64_128_verification.txt"))
    assert _smhasher_verification(lambda x: int(fmix64_np(np.array([x], np.uint64).view(np.int64))[0])) == want


def test_fmix64_zero_is_fixed_point():
    assert oracle.fmix64(0) == 0


def _fmix64_inverse(h):
    inv1 = pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)
    inv2 = pow(0xFF51AFD7ED558CCD, -1, 1 << 64)
    h ^= h >> 33
    h = (h * inv1) & M64
    h ^= h >> 33
    h = (h * inv2) & M64
    h ^= h >> 33
    return h


def test_fmix64_bijective():
    rng = np.random.default_rng(1)
    xs = [int(x) for x in rng.integers(0, 1 << 63, 2000, dtype=np.uint64, endpoint=True)]
    xs += [0, 1, M64, 1 << 63, (1 << 63) - 1]
    for x in xs:
        assert _fmix64_inverse(oracle.fmix64(x)) == x


def test_fmix64_regression(golden_dir):
    with open(os.path.join(golden_dir, "fmix64_regression.txt")) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    ps = [1, 3, 4, 8, 16, 32, 1000]
    for row in lines:
        k = int(row[0])
        assert oracle.fmix64(k & M64) == int(row[1], 16)
        for p, want in zip(ps, row[2:]):
            assert oracle.partition_of(k, p) == int(want)


def test_destination_is_unsigned_remainder():
    # fmix64(INT64_MAX) has its top bit set: a signed remainder would differ
    for k in [(1 << 63) - 1, -(1 << 63), -1, 1]:
        h = oracle.fmix64(k & M64)
        for P in [3, 5, 7, 1000, 4095]:
            assert oracle.partition_of(k, P) == h % P


def test_int32_keys_sign_extend():
    k32 = np.array([-1, -2, 5, -(1 << 31), (1 << 31) - 1], np.int32)
    k64 = k32.astype(np.int64)
    for P in [3, 16, 1000]:
        a = oracle.hash_partition(k32, np.arange(5), P)
        b = oracle.hash_partition(k64, np.arange(5), P)
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        assert a[0].dtype == np.int32 and np.array_equal(a[0].astype(np.int64), b[0])


# --------------------------------------------------------------------------
# partition
# --------------------------------------------------------------------------

def _partition_by_argsort(keys, payload, P):
    dest = np.array([oracle.partition_of(int(k), P) for k in keys], dtype=np.int64)
    order = np.argsort(dest, kind="stable")
    off = np.concatenate([[0], np.cumsum(np.bincount(dest, minlength=P))]).astype(np.int64)
    return keys[order], payload[order], off


@pytest.mark.parametrize("P", [1, 2, 3, 4, 7, 32, 1000, 4096])
def test_partition_matches_stable_argsort(P):
    kl, vl, _, _ = uniform_tables(5000, 0, 3000, seed=P)
    got = oracle.hash_partition(kl, vl, P)
    want = _partition_by_argsort(kl, vl, P)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


@pytest.mark.parametrize("name", ["extremes", "int32_negative", "int32_extremes", "all_equal"])
def test_partition_edge_cases_match_argsort(name):
    kl, vl, kr, vr, _ = edge_tables(name)
    for P in [1, 5, 32]:
        for k, v in [(kl, vl), (kr, vr)]:
            got = oracle.hash_partition(k, v, P)
            want = _partition_by_argsort(k, v, P)
            for g, w in zip(got, want):
                assert np.array_equal(g, w)


def test_partition_empty_and_more_destinations_than_rows():
    ko, vo, off = oracle.hash_partition(np.zeros(0, np.int64), np.zeros(0, np.int64), 8)
    assert ko.size == 0 and vo.size == 0 and np.array_equal(off, np.zeros(9, np.int64))
    k = np.array([10, 20, 30], np.int64)
    ko, vo, off = oracle.hash_partition(k, np.arange(3), 4096)
    assert off[-1] == 3 and np.count_nonzero(np.diff(off)) <= 3
    check_partition_invariants(k, ko, vo, off, 4096, lambda x: part_np(x, 4096))


def test_partition_invariants_plain_workload():
    kl, vl, kr, vr = config_inputs("plain")
    for k, v in [(kl, vl), (kr, vr)]:
        ko, vo, off = oracle.hash_partition(k, v, 4)
        check_partition_invariants(k, ko, vo, off, 4, lambda x: part_np(x, 4))


def test_partition_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.hash_partition(np.zeros(3, np.int64), np.zeros(3, np.int64), 0)


def test_paper_left_partition_counts(golden_dir):
    """The 1E8-row left table is a permutation of [0, 1E8): its destination
    counts are seed-independent.  Checked here on a random permutation of the
    key set (the golden file was written from arange)."""
    with open(os.path.join(golden_dir, "paper_left_partition_counts_p32.txt")) as f:
        want = [int(x) for ln in f if not ln.startswith("#") for x in ln.split()]
    assert sum(want) == 100_000_000
    n = 100_000_000
    keys = np.random.default_rng(7).permutation(n).astype(np.int64)
    cnt = np.bincount(part_np(keys, 32), minlength=32)
    assert cnt.tolist() == want


# --------------------------------------------------------------------------
# join
# --------------------------------------------------------------------------

def test_join_worked_example(golden_dir):
    with open(os.path.join(golden_dir, "join_worked_example.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    kl = np.array([int(x) for x in rows[0][1:]], np.int64)
    kr = np.array([int(x) for x in rows[1][1:]], np.int64)
    want = np.array([[int(x) for x in r[1:]] for r in rows[2:]], np.int64)
    res = oracle.join(kl, np.arange(kl.size), kr, np.arange(kr.size))
    assert res["total"] == len(want)
    got = np.stack([res["key"], res["lpay"], res["rpay"]], axis=1)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(6))
def test_join_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    nl, nr = int(rng.integers(0, 250)), int(rng.integers(0, 250))
    kr_range = int(rng.integers(1, 60))
    kl, vl, kr, vr = uniform_tables(nl, nr, kr_range, seed=seed)
    # shift payloads so that left and right payloads differ
    vl = vl * 3 + 11
    vr = vr * 7 - 5
    res = oracle.join(kl, vl, kr, vr)
    want = brute_force_join(kl, vl, kr, vr)
    assert res["total"] == want[0].size
    for g, w in zip((res["key"], res["lpay"], res["rpay"]), want):
        assert np.array_equal(g, w)


@pytest.mark.parametrize("name", ["empty_left", "empty_right", "both_empty", "extremes",
                                  "int32_negative", "int32_extremes"])
def test_join_edge_cases_match_brute_force(name):
    kl, vl, kr, vr, _ = edge_tables(name)
    kl, kr = kl[:400], kr[:400]
    vl, vr = vl[:400], vr[:400]
    res = oracle.join(kl, vl, kr, vr)
    want = brute_force_join(kl, vl, kr, vr)
    assert res["total"] == want[0].size
    for g, w in zip((res["key"], res["lpay"], res["rpay"]), want):
        assert np.array_equal(g, w)


def test_join_all_equal_keys_is_full_cross_product():
    kl, vl, kr, vr, _ = edge_tables("all_equal")
    res = oracle.join(kl, vl, kr, vr)
    assert res["total"] == kl.size * kr.size
    ll, rr = np.meshgrid(vl, vr, indexing="ij")
    assert np.array_equal(res["lpay"], ll.ravel()) and np.array_equal(res["rpay"], rr.ravel())


def test_join_matches_pandas_plain_workload():
    kl, vl, kr, vr = config_inputs("plain")
    res = oracle.join(kl, vl, kr, vr, P=4)
    m = pd.merge(pd.DataFrame({"k": kl, "l": vl}), pd.DataFrame({"k": kr, "r": vr}),
                 on="k", how="inner")
    want = canonical(m["k"].to_numpy(), m["l"].to_numpy(), m["r"].to_numpy())
    assert res["total"] == want[0].size
    for g, w in zip((res["key"], res["lpay"], res["rpay"]), want):
        assert np.array_equal(g, w)
    # destination counts of the output rows
    assert res["per_part"].sum() == res["total"]
    assert np.array_equal(res["per_part"], np.bincount(part_np(res["key"], 4), minlength=4))


def test_join_matches_pandas_skewed():
    kl, vl, kr, vr = zipf_tables(20_000, 20_000, 1.1, 5_000, seed=3)
    res = oracle.join(kl, vl, kr, vr, P=16)
    m = pd.merge(pd.DataFrame({"k": kl, "l": vl}), pd.DataFrame({"k": kr, "r": vr}),
                 on="k", how="inner")
    assert res["total"] == len(m) == expected_cardinality(kl, kr)
    want = canonical(m["k"].to_numpy(), m["l"].to_numpy(), m["r"].to_numpy())
    for g, w in zip((res["key"], res["lpay"], res["rpay"]), want):
        assert np.array_equal(g, w)


def test_join_match_fraction_closed_form():
    # left keys distinct => every matched right row has exactly one partner,
    # so |J| = round(0.3 * n_right) exactly
    kl, vl, kr, vr = match_fraction_tables(200_000, 150_000, 0.3, seed=5)
    res = oracle.join(kl, vl, kr, vr, P=32)
    assert res["total"] == round(0.3 * 150_000)
    check_join_rows(kl, kr, res["key"], res["lpay"], res["rpay"])
    hit = kr < 200_000
    assert np.array_equal(np.sort(res["rpay"]), np.flatnonzero(hit))


def test_match_counts_brute_force():
    kl, vl, kr, vr = uniform_tables(300, 200, 50, seed=9)
    got = oracle.match_counts(kl, kr)
    want = np.array([int(np.sum(kl == k)) for k in kr], np.int64)
    assert np.array_equal(got, want)
    assert got.sum() == oracle.join(kl, vl, kr, vr, materialize=False)["total"]


# ---- transpose sum (the cuPy benchmark's y = x + x.T) -------------------------------

def _read_example(golden_dir):
    rows = [ln.split() for ln in open(os.path.join(golden_dir, "transpose_sum_example.txt"))
            if ln.strip() and not ln.startswith("#")]
    vals = np.array(rows, dtype=np.float64)
    return vals[:3], vals[3:]


def test_transpose_sum_worked_example(golden_dir):
    x, y = _read_example(golden_dir)
    assert np.array_equal(oracle.transpose_sum(x), y)


def test_transpose_sum_invariants():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((97, 97)) * 10.0 ** rng.integers(-30, 30, (97, 97))
    y = oracle.transpose_sum(x)
    # IEEE addition commutes: the result is symmetric bit for bit
    assert np.array_equal(y.view(np.uint64), y.T.view(np.uint64))
    # the diagonal is doubled exactly (x + x = 2x, no rounding)
    assert np.array_equal(np.diag(y), 2.0 * np.diag(x))
    # x + x^T - x^T recovers x only up to rounding: not the identity map
    assert not np.array_equal(y, x)


def test_transpose_sum_rounding_pin():
    """1 + 2^-53 lies halfway between 1 and the next double: ties to even
    gives 1.0; 1 + 3 2^-53 rounds up to 1 + 2^-51."""
    x = np.array([[0.0, 1.0, 1.0], [2.0 ** -53, 0.0, 0.0], [3 * 2.0 ** -53, 0.0, 0.0]])
    y = oracle.transpose_sum(x)
    assert y[0, 1] == 1.0 and y[1, 0] == 1.0
    assert y[0, 2] == 1.0 + 2.0 ** -51


def test_transpose_sum_edge_shapes():
    assert oracle.transpose_sum(np.zeros((0, 0))).shape == (0, 0)
    assert oracle.transpose_sum(np.array([[2.5]]))[0, 0] == 5.0
    with pytest.raises(ValueError):
        oracle.transpose_sum(np.zeros((2, 3)))


# --------------------------------------------------------------------------
# the threaded CPU baseline (same partition and join over host threads)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("P", [1, 4, 7, 32])
def test_merge_threads_partitions_equal_stable_argsort(threads, P):
    kl, vl, kr, vr = uniform_tables(3000, 2500, 1500, seed=P * 10 + threads)
    res = oracle.merge_threads(kl, vl, kr, vr, P, threads)
    for side, (k, v) in (("left", (kl, vl)), ("right", (kr, vr))):
        want = _partition_by_argsort(k, v, P)
        for g, w in zip(res[side], want):
            assert np.array_equal(g, w)


@pytest.mark.parametrize("threads", [1, 2, 5, 16])
def test_merge_threads_join_equals_brute_force(threads):
    kl, vl, kr, vr = uniform_tables(300, 280, 40, seed=threads)
    vl, vr = vl * 3 + 11, vr * 7 - 5
    res = oracle.merge_threads(kl, vl, kr, vr, 4, threads, cap=kl.size * kr.size)
    want = brute_force_join(kl, vl, kr, vr)
    assert res["total"] == want[0].size
    for g, w in zip(canonical(res["key"], res["lpay"], res["rpay"]), want):
        assert np.array_equal(g, w)
    # destination p's rows sit at [out_off[p], out_off[p+1])
    off = res["out_off"]
    for p in range(4):
        assert (part_np(res["key"][off[p]:off[p + 1]], 4) == p).all()


def test_merge_threads_plain_workload_and_edges():
    kl, vl, kr, vr = config_inputs("plain")
    res = oracle.merge_threads(kl, vl, kr, vr, 4, 8)
    ref = oracle.join(kl, vl, kr, vr, P=4)
    assert res["total"] == ref["total"]
    assert np.array_equal(np.diff(res["out_off"]), ref["per_part"])
    for g, w in zip(canonical(res["key"], res["lpay"], res["rpay"]),
                    (ref["key"], ref["lpay"], ref["rpay"])):
        assert np.array_equal(g, w)
    for name in ["empty_left", "both_empty", "all_equal", "int32_negative", "extremes"]:
        kl, vl, kr, vr, _ = edge_tables(name)
        kl, vl, kr, vr = kl[:300], vl[:300], kr[:300], vr[:300]
        res = oracle.merge_threads(kl, vl, kr, vr, 5, 4, cap=kl.size * kr.size)
        want = brute_force_join(kl, vl, kr, vr)
        assert res["total"] == want[0].size, name
        for g, w in zip(canonical(res["key"], res["lpay"], res["rpay"]), want):
            assert np.array_equal(g, w), name


def test_merge_threads_small_capacity_writes_offsets_only():
    kl, vl, kr, vr = uniform_tables(500, 500, 50, seed=1)
    want = expected_cardinality(kl, kr)
    res = oracle.merge_threads(kl, vl, kr, vr, 4, 4, cap=want - 1)
    assert res["total"] == want and res["out_off"][-1] == want and "key" not in res
