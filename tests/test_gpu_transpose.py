"""Parity of mdx_transpose_sum (y = x + x^T, float64) with the oracle:
bit-exact, ragged edges, in place, and the RI2 benchmark size."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _matrix(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, n)) * 10.0 ** rng.integers(-12, 12, (n, n))
    if n >= 4:  # signed zeros, infinities, subnormals
        x[0, 1], x[1, 0] = -0.0, 0.0
        x[2, 3], x[3, 2] = np.inf, 1.0
        x[1, 3], x[3, 1] = 5e-324, -5e-324
    return x


def _same_bits(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


@pytest.mark.parametrize("n", [1, 2, 7, 63, 64, 65, 200, 1000, 4097])
def test_transpose_sum_matches_oracle(n):
    import paper_2101_08878_amd as mdx
    announce(f"transpose sum n={n}")
    x = _matrix(n, n)
    y = mdx.mdx_transpose_sum(dev(x))
    torch.cuda.synchronize()
    assert _same_bits(host(y), oracle.transpose_sum(x))


@pytest.mark.parametrize("n", [129, 2048])
def test_transpose_sum_in_place(n):
    import paper_2101_08878_amd as mdx
    announce(f"transpose sum in place n={n}")
    x = _matrix(n, 17)
    t = dev(x)
    mdx.mdx_transpose_sum(t, out=t)
    torch.cuda.synchronize()
    assert _same_bits(host(t), oracle.transpose_sum(x))


def test_transpose_sum_benchmark_size():
    """16K x 16K, the RI2 benchmark's array (2 GiB): full comparison."""
    import paper_2101_08878_amd as mdx
    announce("transpose sum 16384")
    n = 16384
    rng = np.random.default_rng(0)
    x = rng.random((n, n))
    y = mdx.mdx_transpose_sum(dev(x))
    torch.cuda.synchronize()
    assert _same_bits(host(y), oracle.transpose_sum(x))
