"""Parity of mdx_merge (partition both tables, join every partition in
cache-sized groups) with the oracle, plus the 1E8 x 1E8 workload in the
launch configuration the benchmark times, checked through properties that
hold at any size."""

import numpy as np
import pytest

import oracle
from tests.gpu_util import announce, assert_join_equals_oracle, require_gpu, run_merge
from tests.helpers import part_np
from workloads import config_inputs, match_fraction_tables, zipf_tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("group", [0, 1, 3, 4])
def test_merge_plain_workload(group):
    announce(f"merge plain group={group}")
    kl, vl, kr, vr = config_inputs("plain")
    got = run_merge(kl, vl, kr, vr, 4, group=group)
    assert_join_equals_oracle(kl, vl, kr, vr, 4, got)


@pytest.mark.parametrize("group", [0, 1, 5, 32])
def test_merge_paper_shape_reduced(group):
    """The 1E8 workload's generator at 2E6 rows per side, P = 32."""
    announce(f"merge paper x0.02 group={group}")
    kl, vl, kr, vr = config_inputs("paper", scale=0.02)
    got = run_merge(kl, vl, kr, vr, 32, group=group)
    assert_join_equals_oracle(kl, vl, kr, vr, 32, got)


def test_merge_int32_keys():
    announce("merge int32")
    kl, vl, kr, vr = match_fraction_tables(300_000, 250_000, 0.3, seed=4, key_dtype=np.int32)
    got = run_merge(kl, vl, kr, vr, 8, group=2)
    assert_join_equals_oracle(kl, vl, kr, vr, 8, got)


def test_merge_skewed_reduced():
    announce("merge zipf reduced")
    kl, vl, kr, vr = zipf_tables(15_000, 15_000, 1.1, 10_000, seed=0)
    total = oracle.join(kl, vl, kr, vr, materialize=False)["total"]
    got = run_merge(kl, vl, kr, vr, 16, cap=total, group=3)
    assert_join_equals_oracle(kl, vl, kr, vr, 16, got)


def test_merge_paper_scale_properties():
    """1E8 x 1E8, P = 32, default grouping (what the benchmark times).

    Left keys are a permutation of [0, 1E8), so a right row matches iff its
    key is below 1E8, and then exactly once: the output must be exactly the
    right rows with key < 1E8, each paired with the unique left row holding
    its key (payload = row index), |J| = 3E7, and partition p's block must
    hold exactly the output keys with destination p."""
    announce("merge paper scale 1e8")
    n = 100_000_000
    kl, vl, kr, vr = config_inputs("paper")
    got = run_merge(kl, vl, kr, vr, 32, cap=n)
    assert got["status"] == 0
    off = got["off"]
    total = int(off[-1])
    assert total == 30_000_000
    key, lp, rp = got["key"][:total], got["lpay"][:total], got["rpay"][:total]
    # every output row is a genuine match
    assert np.array_equal(kl[lp], key)
    assert np.array_equal(kr[rp], key)
    # completeness and no duplicates: the right payloads are exactly the hits
    hits = np.flatnonzero(kr < n)
    assert hits.size == total
    assert np.array_equal(np.sort(rp), hits)
    # partition blocks
    dest = np.repeat(np.arange(32), np.diff(off))
    assert np.array_equal(part_np(key, 32), dest)
