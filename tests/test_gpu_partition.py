"""Parity of mdx_hash_partition with the oracle's stable counting sort.

The partition result is unique, so outputs are compared byte for byte."""

import os

import numpy as np
import pytest

import oracle
from tests.gpu_util import announce, require_gpu, run_partition
from workloads import config_inputs, edge_tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _assert_same(keys, pay, P):
    got = run_partition(keys, pay, P)
    want = oracle.hash_partition(keys, pay, P)
    assert got[0].dtype == keys.dtype
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


# 3 * 4096 + 123 rows: several tiles of both tile sizes plus a ragged tail
N_RAGGED = 3 * 4096 + 123


@pytest.mark.parametrize("P", [1, 2, 3, 7, 32, 255, 256, 257, 1000, 4096])
@pytest.mark.parametrize("dtype", [np.int64, np.int32])
def test_partition_ragged_matches_oracle(P, dtype):
    announce(f"partition ragged P={P} dtype={np.dtype(dtype).name}")
    rng = np.random.default_rng(P)
    info = np.iinfo(dtype)
    keys = rng.integers(info.min, info.max, N_RAGGED, dtype=np.int64, endpoint=True).astype(dtype)
    _assert_same(keys, np.arange(N_RAGGED, dtype=np.int64), P)


@pytest.mark.parametrize("P", [1, 2, 4])
@pytest.mark.parametrize("dtype", [np.int64, np.int32])
def test_partition_few_destinations_many_tiles(P, dtype):
    """At most 4 destinations the histogram counts by wave ballots: 1E6 rows
    (245 tiles and a ragged tail) byte-exact against the oracle."""
    announce(f"partition few destinations P={P} dtype={np.dtype(dtype).name}")
    n = 1_000_000
    info = np.iinfo(dtype)
    keys = np.random.default_rng(100 + P).integers(info.min, info.max, n, dtype=np.int64,
                                                  endpoint=True).astype(dtype)
    _assert_same(keys, np.arange(n, dtype=np.int64), P)


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4095, 4096, 4097])
def test_partition_small_sizes(n):
    announce(f"partition n={n}")
    keys = np.random.default_rng(n).integers(0, 50, n).astype(np.int64)
    for P in [1, 4, 33, 300]:
        _assert_same(keys, np.arange(n, dtype=np.int64) * 3 - 7, P)


@pytest.mark.parametrize("name", ["extremes", "int32_negative", "int32_extremes", "all_equal"])
def test_partition_edge_tables(name):
    announce(f"partition edge {name}")
    kl, vl, kr, vr, _ = edge_tables(name)
    for P in [1, 5, 32, 4096]:
        _assert_same(kl, vl, P)
        _assert_same(kr, vr, P)


def test_partition_plain_workload():
    announce("partition plain workload")
    kl, vl, kr, vr = config_inputs("plain")
    _assert_same(kl, vl, 4)
    _assert_same(kr, vr, 4)


def test_partition_is_deterministic():
    announce("partition determinism")
    kl, vl, _, _ = config_inputs("paper", scale=0.01)
    a = run_partition(kl, vl, 32)
    b = run_partition(kl, vl, 32)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_partition_paper_scale_bit_exact(golden_dir):
    """1E8-row left and right tables, P = 32: byte-exact against the oracle,
    and the left table's per-destination counts equal the seed-independent
    golden counts."""
    announce("partition paper scale 1e8")
    kl, vl, kr, vr = config_inputs("paper")
    with open(os.path.join(golden_dir, "paper_left_partition_counts_p32.txt")) as f:
        counts = [int(x) for ln in f if not ln.startswith("#") for x in ln.split()]
    got = run_partition(kl, vl, 32)
    assert np.diff(got[2]).tolist() == counts
    want = oracle.hash_partition(kl, vl, 32)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    del got, want
    got = run_partition(kr, vr, 32)
    want = oracle.hash_partition(kr, vr, 32)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


@pytest.mark.parametrize("dtype", [np.int64, np.int32])
@pytest.mark.parametrize("shift", [1, 2, 3])
def test_partition_key_column_not_16_byte_aligned(dtype, shift):
    """A key column that starts 4, 8 or 12 bytes past a 16-byte boundary (a
    slice of a larger column): the histogram cannot read it 16 bytes per
    lane and must take the per-row path, with the same result."""
    import torch

    import paper_2101_08878_amd as mdx
    from tests.gpu_util import host

    itemsize = np.dtype(dtype).itemsize
    if (shift * 4) % itemsize:
        pytest.skip("offset not a multiple of the key width")
    skip = shift * 4 // itemsize
    announce(f"partition unaligned keys {np.dtype(dtype).name} +{shift * 4} B")
    n = N_RAGGED
    keys = np.random.default_rng(40 + shift).integers(-10**6, 10**6, n + skip).astype(dtype)
    pay = np.arange(n, dtype=np.int64)
    base = torch.from_numpy(keys).to("cuda")
    assert base.data_ptr() % 16 == 0
    kd = base[skip:]
    assert kd.data_ptr() % 16 != 0
    for P in [3, 7, 32]:  # 3: the few-destination histogram on the per-row path
        ko, vo, off = mdx.mdx_hash_partition(kd, torch.from_numpy(pay).to("cuda"), P)
        torch.cuda.synchronize()
        want = oracle.hash_partition(keys[skip:], pay, P)
        for g, w in zip((host(ko), host(vo), host(off)), want):
            assert np.array_equal(g, w)
