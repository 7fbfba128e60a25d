"""Serving (mdx_server_*): merges admitted while others run.

Each result must be the same in the mix as alone (tolerance 0: identical
rows after canonical ordering, identical offsets and status) and equal to
the oracle; the memory budget must hold at every admission."""

import numpy as np
import pytest
import torch

from tests.gpu_util import announce, assert_join_equals_oracle, dev, host, require_gpu, run_merge
from tests.helpers import canonical
from workloads import match_fraction_tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _requests(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nl = int(round(np.exp(rng.uniform(np.log(1e3), np.log(3e5)))))
        nr = int(round(np.exp(rng.uniform(np.log(1e3), np.log(3e5)))))
        f = float(rng.uniform(0.1, 0.9))
        kl, vl, kr, vr = match_fraction_tables(nl, nr, f, seed=int(rng.integers(1 << 30)))
        out.append((kl, vl, kr, vr, 8))
    return out


def _job(kl, vl, kr, vr, P):
    import paper_2101_08878_amd as mdx
    return mdx.MergeJob(dev(kl), dev(vl), dev(kr), dev(vr), P, max(kr.size, 1),
                        status=torch.zeros(1, dtype=torch.int32, device="cuda"))


def _serve(server, jobs):
    """Submit in order; when busy, poll until the head is admitted."""
    pending, done = list(range(len(jobs))), []
    while pending or len(done) < len(jobs):
        while pending:
            if server.submit(jobs[pending[0]], pending[0]) is None:
                break
            pending.pop(0)
        done += server.poll()
    return done


def test_server_mix_equals_alone():
    import paper_2101_08878_amd as mdx
    announce("server: 40 requests, 4 slots")
    reqs = _requests(40, seed=5)
    jobs = [_job(*r) for r in reqs]
    with mdx.Server(4, 300_000, 300_000, 8, 1 << 34) as srv:
        done = _serve(srv, jobs)
        assert sorted(done) == list(range(len(jobs)))
        assert srv.stats() == (0, 0)
    torch.cuda.synchronize()
    for i, ((kl, vl, kr, vr, P), j) in enumerate(zip(reqs, jobs)):
        total = int(j.out_offsets[-1].item())
        mix = dict(key=host(j.out[0]), lpay=host(j.out[1]), rpay=host(j.out[2]),
                   off=host(j.out_offsets), status=int(j.status.item()), cap=j.out_capacity)
        alone = run_merge(kl, vl, kr, vr, P, cap=j.out_capacity)
        assert np.array_equal(mix["off"], alone["off"]), i
        assert mix["status"] == alone["status"] == 0, i
        for a, b in zip(canonical(mix["key"][:total], mix["lpay"][:total], mix["rpay"][:total]),
                        canonical(alone["key"][:total], alone["lpay"][:total], alone["rpay"][:total])):
            assert np.array_equal(a, b), i
        assert_join_equals_oracle(kl, vl, kr, vr, P, mix)


def test_server_budget_admission():
    """A budget of about two requests: a third is refused while two run, even
    with slots free, and the bytes in flight never exceed the budget."""
    import paper_2101_08878_amd as mdx
    announce("server: budget admission")
    reqs = [match_fraction_tables(200_000, 200_000, 0.5, seed=s) + (8,) for s in range(6)]
    jobs = [_job(*r) for r in reqs]
    one = 2 * 200_000 * 16 + 200_000 * 24 + 9 * 8
    budget = 2 * one + one // 2
    with mdx.Server(4, 200_000, 200_000, 8, budget) as srv:
        assert srv.submit(jobs[0], 0) is not None
        assert srv.submit(jobs[1], 1) is not None
        busy, inflight = srv.stats()
        assert busy == 2 and inflight == 2 * one
        # finished merges count until they are polled: the third must wait
        assert srv.submit(jobs[2], 2) is None
        pending, done = list(range(2, len(jobs))), []
        while pending or len(done) < len(jobs):
            while pending and srv.submit(jobs[pending[0]], pending[0]) is not None:
                pending.pop(0)
                assert srv.stats()[1] <= budget
            done += srv.poll()
        assert sorted(done) == list(range(len(jobs)))
    torch.cuda.synchronize()
    for (kl, vl, kr, vr, P), j in zip(reqs, jobs):
        got = dict(key=host(j.out[0]), lpay=host(j.out[1]), rpay=host(j.out[2]),
                   off=host(j.out_offsets), status=int(j.status.item()), cap=j.out_capacity)
        assert_join_equals_oracle(kl, vl, kr, vr, P, got)


def _tables_and_probes(seed):
    """Three build tables to keep on the device (in one every key appears 4
    times) and 30 probe requests against them, each with its own match
    fraction drawn from U[0.1, 0.9]."""
    rng = np.random.default_rng(seed)
    tables = []
    for n, P in [(250_000, 8), (40_000, 8), (120_000, 5)]:
        kl = rng.permutation(n).astype(np.int64)
        if n == 120_000:
            kl = (kl % 30_000).astype(np.int64)  # every key 4 times
        tables.append((kl, np.arange(n, dtype=np.int64) * 3 + 1, P))
    probes = []
    for i in range(30):
        t = int(rng.integers(0, len(tables)))
        kl = tables[t][0]
        nr = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e5)))))
        f = float(rng.uniform(0.1, 0.9))
        m = int(round(f * nr))
        hit = kl[rng.integers(0, kl.size, m)]
        miss = rng.integers(1 << 40, 1 << 41, nr - m)
        kr = np.concatenate([hit, miss])[rng.permutation(nr)].astype(np.int64)
        probes.append((t, kr, np.arange(nr, dtype=np.int64) * 7 - 2))
    return tables, probes


def test_server_probes_of_resident_tables_equal_alone():
    """Build tables once (mdx_join_build), then admit probe requests against
    them into 4 slots: each result equals the same probe run alone
    (mdx_hash_partition + mdx_join_probe) and the oracle."""
    import paper_2101_08878_amd as mdx
    announce("server: 30 probes of 3 resident tables, 4 slots")
    tables, probes = _tables_and_probes(11)
    built = []
    for kl, vl, P in tables:
        lk, lv, lo = mdx.mdx_hash_partition(dev(kl), dev(vl), P)
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        built.append(mdx.mdx_join_build(lk, lv, lo, P, status=st))
        torch.cuda.synchronize()
        assert int(st.item()) == 0
    jobs = []
    for t, kr, vr in probes:
        cap = int(kr.size) * (4 if t == 2 else 1)
        jobs.append(mdx.ProbeJob(built[t], dev(kr), dev(vr), cap,
                                 status=torch.zeros(1, dtype=torch.int32, device="cuda")))
    pending, done = list(range(len(jobs))), []
    with mdx.Server(4, 300_000, 300_000, 8, 1 << 34) as srv:
        while pending or len(done) < len(jobs):
            while pending and srv.submit_probe(jobs[pending[0]], pending[0]) is not None:
                pending.pop(0)
            done += srv.poll()
        assert sorted(done) == list(range(len(jobs)))
        assert srv.stats() == (0, 0)
    torch.cuda.synchronize()
    for i, ((t, kr, vr), j) in enumerate(zip(probes, jobs)):
        kl, vl, P = tables[t]
        total = int(j.out_offsets[-1].item())
        assert int(j.status.item()) == 0, i
        mix = dict(key=host(j.out[0]), lpay=host(j.out[1]), rpay=host(j.out[2]),
                   off=host(j.out_offsets), status=0, cap=j.out_capacity)
        rk, rv, ro = mdx.mdx_hash_partition(dev(kr), dev(vr), P)
        ok, ol, orr, off = mdx.mdx_join_probe(built[t], rk, rv, ro, out_capacity=j.out_capacity)
        torch.cuda.synchronize()
        assert np.array_equal(mix["off"], host(off)), i
        for a, b in zip(canonical(mix["key"][:total], mix["lpay"][:total], mix["rpay"][:total]),
                        canonical(host(ok)[:total], host(ol)[:total], host(orr)[:total])):
            assert np.array_equal(a, b), i
        assert_join_equals_oracle(kl, vl, kr, vr, P, mix)


def test_server_probe_rejects_what_it_cannot_admit():
    """Host checks of a probe request: a probe beyond the server's limits and
    a table of a larger P are refused with MDX_ERR_INVALID, nothing runs."""
    import paper_2101_08878_amd as mdx
    announce("server: probe limits")
    kl = np.arange(1000, dtype=np.int64)
    lk, lv, lo = mdx.mdx_hash_partition(dev(kl), dev(kl), 16)
    t16 = mdx.mdx_join_build(lk, lv, lo, 16)
    kr = dev(np.arange(5000, dtype=np.int64))
    with mdx.Server(2, 2000, 2000, 8, 1 << 30) as srv:
        with pytest.raises(mdx.MdxError):
            srv.submit_probe(mdx.ProbeJob(t16, kr[:100], kr[:100], 100), 0)  # P = 16 > max_P
        lk8, lv8, lo8 = mdx.mdx_hash_partition(dev(kl), dev(kl), 8)
        t8 = mdx.mdx_join_build(lk8, lv8, lo8, 8)
        with pytest.raises(mdx.MdxError):
            srv.submit_probe(mdx.ProbeJob(t8, kr, kr, 5000), 1)  # n > max_right
        assert srv.stats() == (0, 0)
    torch.cuda.synchronize()
