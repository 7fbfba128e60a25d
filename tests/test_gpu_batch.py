"""Parity of mdx_merge_batch (many merges in one call) with the oracle.

Every merge of a batch must equal what the oracle computes for it (rows
after canonical ordering, per-partition offsets exact), whatever the number
of lanes, and a batch captured into a HIP graph must give the same result
on every replay."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import announce, assert_join_equals_oracle, dev, host, require_gpu
from workloads import batch_specs, batch_tables, edge_tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _batch_inputs():
    """A mixed batch: log-uniform sizes (some below one tile), both key
    widths, several P, empty sides, and one merge whose repeated key sends
    the device to the global-table fallback."""
    items = []
    for s in batch_specs(36, seed=11, lo=1, hi=2e5):
        kl, vl, kr, vr = batch_tables(s, seed=11)
        items.append((kl, vl, kr, vr, [1, 3, 8, 32][s.index % 4]))
    for name in ["empty_left", "empty_right", "both_empty", "int32_negative"]:
        kl, vl, kr, vr, _ = edge_tables(name)
        items.append((kl, vl, kr, vr, 5))
    kl = np.full(20000, 5, np.int64)
    kr = np.concatenate([np.full(300, 5, np.int64), np.arange(10, 5000, dtype=np.int64)])
    items.append((kl, np.arange(kl.size, dtype=np.int64), kr, np.arange(kr.size, dtype=np.int64), 4))
    return items


def _jobs(items):
    import paper_2101_08878_amd as mdx
    jobs = []
    for kl, vl, kr, vr, P in items:
        cap = max(oracle.join(kl, vl, kr, vr, materialize=False)["total"], 1)
        jobs.append(mdx.MergeJob(dev(kl), dev(vl), dev(kr), dev(vr), P, cap,
                                 status=torch.zeros(1, dtype=torch.int32, device="cuda")))
    return jobs


def _check(items, jobs):
    for i, ((kl, vl, kr, vr, P), j) in enumerate(zip(items, jobs)):
        got = dict(key=host(j.out[0]), lpay=host(j.out[1]), rpay=host(j.out[2]),
                   off=host(j.out_offsets), status=int(j.status.item()), cap=j.out_capacity)
        try:
            assert_join_equals_oracle(kl, vl, kr, vr, P, got)
        except AssertionError as e:
            raise AssertionError(f"merge {i} (nL={kl.size}, nR={kr.size}, P={P}): {e}") from e


@pytest.mark.parametrize("lanes", [1, 3, 8])
def test_batch_matches_oracle(lanes):
    import paper_2101_08878_amd as mdx
    announce(f"merge batch lanes={lanes}")
    items = _batch_inputs()
    jobs = _jobs(items)
    mdx.mdx_merge_batch(jobs, lanes=lanes)
    torch.cuda.synchronize()
    _check(items, jobs)


def test_batch_single_and_empty():
    import paper_2101_08878_amd as mdx
    announce("merge batch of one and of none")
    items = _batch_inputs()[:1]
    jobs = _jobs(items)
    mdx.mdx_merge_batch(jobs, lanes=4)
    torch.cuda.synchronize()
    _check(items, jobs)
    assert mdx.mdx_merge_batch([], lanes=4) == []


def test_batch_graph_replays():
    """Capture one batch (4 lanes) into a graph; replay it three times,
    clearing the outputs with eager work in between, and check every
    replay against the oracle."""
    import paper_2101_08878_amd as mdx
    announce("merge batch in a HIP graph")
    items = _batch_inputs()
    jobs = _jobs(items)
    ws = torch.empty(mdx.mdx_merge_batch_workspace_bytes(jobs, 4), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        mdx.mdx_merge_batch(jobs, lanes=4, workspace=ws, stream=s)  # lanes exist before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        mdx.mdx_merge_batch(jobs, lanes=4, workspace=ws, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for j in jobs:
            for t in j.out:
                t.fill_(-1)
            j.out_offsets.fill_(-1)
            j.status.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check(items, jobs)


def test_batch_config4_subset():
    """The first 16 merges of the 4096-merge batch at their real sizes (up to
    4E6 rows per side, P = 8), 4 lanes."""
    import paper_2101_08878_amd as mdx
    announce("merge batch: first 16 merges of the 4096-merge batch")
    items = [(*batch_tables(s), 8) for s in batch_specs(4096)[:16]]
    jobs = _jobs(items)
    mdx.mdx_merge_batch(jobs, lanes=4)
    torch.cuda.synchronize()
    _check(items, jobs)


# ---- fused batches (mdx_batch_*) ---------------------------------------------------------

FUSED_TUNINGS = [None, {"fill": 0.5, "fanout": 32, "part_rows": 2},
                 {"fill": 1.0, "fanout": 256, "part_rows": 8}]


@pytest.mark.parametrize("tuning", FUSED_TUNINGS, ids=["default", "small", "full-tables"])
def test_fused_batch_matches_oracle(tuning):
    """Every merge of the mixed batch; fill 1.0 leaves many build sub-buckets
    larger than a table, so they take the chunked join, as the merge with
    20000 copies of one key does under every tuning."""
    import paper_2101_08878_amd as mdx
    announce(f"fused batch tuning={tuning}")
    items = _batch_inputs()
    jobs = _jobs(items)
    fb = mdx.FusedBatch(jobs, tuning=tuning)
    waves, launches = fb.info()
    assert waves == 1 and 0 < launches < 40
    fb.run()
    torch.cuda.synchronize()
    _check(items, jobs)
    fb.close()


def test_fused_batch_in_many_waves():
    """The least workspace: every wave holds as many merges as fit; the
    result does not depend on the waves."""
    import paper_2101_08878_amd as mdx
    announce("fused batch, least workspace")
    items = _batch_inputs()
    jobs = _jobs(items)
    lo, hi = mdx.mdx_batch_workspace_bytes(jobs)
    fb = mdx.FusedBatch(jobs, workspace_bytes=lo)
    waves, _ = fb.info()
    assert waves > 1
    fb.run()
    torch.cuda.synchronize()
    _check(items, jobs)
    fb.close()


def test_fused_batch_overflow_and_chunks():
    """A repeated key whose output exceeds the capacity: the chunked join
    counts it exactly and reports the overflow; the merge beside it is
    unaffected."""
    import paper_2101_08878_amd as mdx
    announce("fused batch: output overflow in the chunked join")
    kl = np.concatenate([np.full(9000, 7, np.int64), np.arange(100, 20000, dtype=np.int64)])
    kr = np.concatenate([np.full(40, 7, np.int64), np.arange(0, 30000, 3, dtype=np.int64)])
    items = [(kl, np.arange(kl.size, dtype=np.int64), kr, np.arange(kr.size, dtype=np.int64), 4)]
    items.append(_batch_inputs()[0])
    jobs = _jobs(items)
    total = jobs[0].out_capacity
    jobs[0].out_capacity = total - 1
    mdx.FusedBatch(jobs).run()
    torch.cuda.synchronize()
    assert int(jobs[0].status.item()) & mdx.MDX_DEV_OUTPUT_OVERFLOW
    ref = oracle.join(*items[0][:4], P=4, materialize=False)
    off = host(jobs[0].out_offsets)
    assert off[-1] == ref["total"] == total
    assert np.array_equal(np.diff(off), ref["per_part"])
    _check(items[1:], jobs[1:])


def test_fused_batch_one_key_at_table_size():
    """Merges whose build side is one key repeated b times, around the fused
    batch's LDS table (3840 rows) and twice it: at most one table the
    sub-bucket is joined at once, beyond it in table-sized chunks."""
    import paper_2101_08878_amd as mdx
    announce("fused batch one key at table size")
    items = []
    for b in [3839, 3840, 3841, 7680, 7681]:
        kl = np.full(b, 9, np.int64)
        kr = np.concatenate([np.full(2, 9, np.int64), np.arange(20, 900, dtype=np.int64)])
        items.append((kl, np.arange(b, dtype=np.int64), kr, np.arange(kr.size, dtype=np.int64),
                      2))
    jobs = _jobs(items)
    fb = mdx.FusedBatch(jobs)
    fb.run()
    torch.cuda.synchronize()
    _check(items, jobs)
    fb.close()


def test_fused_batch_graph_replays():
    """The batch captured into a graph (the plan's copy to the device and
    every launch); three replays with eager clearing in between, each checked
    against the oracle."""
    import paper_2101_08878_amd as mdx
    announce("fused batch in a HIP graph")
    items = _batch_inputs()
    jobs = _jobs(items)
    fb = mdx.FusedBatch(jobs)
    s = torch.cuda.Stream()
    fb.run(s)  # kernels' attributes are set before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fb.run(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for j in jobs:
            for t in j.out:
                t.fill_(-1)
            j.out_offsets.fill_(-1)
            j.status.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check(items, jobs)
    del g
    fb.close()


def test_fused_batch_config4_subset():
    """The first 16 merges of the 4096-merge batch at their real sizes, with
    the tuning table."""
    import paper_2101_08878_amd as mdx
    announce("fused batch: first 16 merges of the 4096-merge batch")
    items = [(*batch_tables(s), 8) for s in batch_specs(4096)[:16]]
    jobs = _jobs(items)
    fb = mdx.FusedBatch(jobs, tuning="table")
    fb.run()
    torch.cuda.synchronize()
    _check(items, jobs)
    fb.close()


def test_fused_batch_many_small_merges():
    """8500 merges of 0 to 60 rows (about 4250 per key width, so each launch
    covers more merges than two 64-way rounds of the block-range search
    resolve: three rounds), empty sides, P from 1 to 9."""
    import paper_2101_08878_amd as mdx
    announce("fused batch: 8500 small merges")
    rng = np.random.default_rng(5)
    items = []
    for i in range(8500):
        nl, nr = int(rng.integers(0, 61)), int(rng.integers(0, 61))
        kd = np.int32 if i % 2 else np.int64
        kl = rng.integers(-20, 20, nl).astype(kd)
        kr = rng.integers(-20, 20, nr).astype(kd)
        items.append((kl, np.arange(nl, dtype=np.int64), kr, np.arange(nr, dtype=np.int64),
                      int(rng.integers(1, 10))))
    jobs = _jobs(items)
    fb = mdx.FusedBatch(jobs)
    fb.run()
    torch.cuda.synchronize()
    _check(items, jobs)
    fb.close()


@pytest.mark.parametrize("P", [300, 4096])
def test_fused_batch_many_partitions(P):
    """More than 256 destinations in the first pass: 1024-row tiles, with a
    merge of the default shape beside it in the same wave."""
    import paper_2101_08878_amd as mdx
    announce(f"fused batch: P={P}")
    items = []
    for s in batch_specs(3, seed=3, lo=1e3, hi=3e5):
        kl, vl, kr, vr = batch_tables(s, seed=3)
        items.append((kl, vl, kr, vr, P))
    kl, vl, kr, vr = batch_tables(batch_specs(1, seed=4, lo=1e4, hi=1e5)[0], seed=4)
    items.append((kl, vl, kr, vr, 8))
    jobs = _jobs(items)
    fb = mdx.FusedBatch(jobs, tuning=[{}, {"part_rows": 8}, {"fanout": 4096}, {}])
    fb.run()
    torch.cuda.synchronize()
    _check(items, jobs)
    fb.close()
