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
