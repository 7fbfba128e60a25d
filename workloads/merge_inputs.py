"""Seeded table generators (numpy PCG64 via ``default_rng``).

Every table is a pair of columns: ``keys`` (int64, or int32 where asked) and
``payload`` (int64) with ``payload[i] == i`` (the original row index).  Draws
happen in a fixed order so that a (generator, seed, sizes) triple always
produces the same bytes.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class WorkloadSpec:
    name: str
    n_left: int
    n_right: int
    P: int
    kind: str          # "uniform" | "match" | "zipf"
    key_dtype: str = "int64"
    key_range: int = 0     # uniform: keys in [0, key_range)
    frac: float = 0.0      # match: fraction of right rows drawn from left keys
    zipf_s: float = 0.0    # zipf: exponent
    zipf_support: int = 0  # zipf: keys in [1, support]
    seed: int = 0


# The single-GPU workloads.  "paper" is one Dask worker's share of the cuDF
# merge at the paper's chunk size (1E8 rows per table, match fraction 0.3),
# partitioned for 32 destination workers (the largest worker count the paper
# runs, Section V-C).
CONFIGS = {
    "plain": WorkloadSpec("plain", 100_000, 100_000, 4, "uniform", key_range=200_000),
    "paper": WorkloadSpec("paper", 100_000_000, 100_000_000, 32, "match", frac=0.3),
    "skewed": WorkloadSpec("skewed", 50_000_000, 50_000_000, 16, "zipf",
                           zipf_s=1.1, zipf_support=10_000_000),
}


def _payload(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.int64)


def uniform_tables(n_left: int, n_right: int, key_range: int, seed: int = 0,
                   key_dtype=np.int64):
    """Keys uniform in [0, key_range), left drawn first, then right."""
    rng = np.random.default_rng(seed)
    kl = rng.integers(0, key_range, n_left, dtype=np.int64).astype(key_dtype)
    kr = rng.integers(0, key_range, n_right, dtype=np.int64).astype(key_dtype)
    return kl, _payload(n_left), kr, _payload(n_right)


def match_fraction_tables(n_left: int, n_right: int, frac: float, seed: int = 0,
                          key_dtype=np.int64):
    """Left keys: a random permutation of [0, n_left) (all distinct).

    Right keys: exactly M = round(frac * n_right) rows take a key drawn
    uniformly (with replacement) from the left keys; the other n_right - M
    rows take keys uniform in [n_left, 2 n_left), which never match.  Row
    positions are then shuffled.  This is the reading of the paper's
    "fraction match" used throughout: the fraction of right rows that find a
    partner.
    """
    rng = np.random.default_rng(seed)
    kl = rng.permutation(n_left).astype(np.int64)
    m = int(round(frac * n_right))
    if n_left > 0:
        hit = kl[rng.integers(0, n_left, m, dtype=np.int64)]
        miss = rng.integers(n_left, 2 * n_left, n_right - m, dtype=np.int64)
    else:
        hit = np.zeros(0, np.int64)
        miss = rng.integers(0, 1 << 40, n_right - m, dtype=np.int64)
    kr = np.concatenate([hit, miss])[rng.permutation(n_right)]
    return kl.astype(key_dtype), _payload(n_left), kr.astype(key_dtype), _payload(n_right)


def zipf_tables(n_left: int, n_right: int, s: float, support: int, seed: int = 0,
                key_dtype=np.int64):
    """Keys Zipf(s) on {1..support}: P(k) proportional to k**-s.

    Inverse-CDF sampling in float64; left drawn first, then right.
    """
    rng = np.random.default_rng(seed)
    w = np.arange(1, support + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def draw(n):
        u = rng.random(n)
        k = 1 + np.searchsorted(cdf, u, side="right")
        return np.minimum(k, support).astype(np.int64)

    kl = draw(n_left)
    kr = draw(n_right)
    return kl.astype(key_dtype), _payload(n_left), kr.astype(key_dtype), _payload(n_right)


def edge_tables(name: str, seed: int = 0):
    """Small adversarial tables: (kL, vL, kR, vR, key_dtype)."""
    rng = np.random.default_rng(seed)
    i64 = np.iinfo(np.int64)
    if name == "empty_left":
        kl = np.zeros(0, np.int64)
        kr = rng.integers(0, 10, 100, dtype=np.int64)
    elif name == "empty_right":
        kl = rng.integers(0, 10, 100, dtype=np.int64)
        kr = np.zeros(0, np.int64)
    elif name == "both_empty":
        kl = np.zeros(0, np.int64)
        kr = np.zeros(0, np.int64)
    elif name == "all_equal":
        kl = np.full(300, 7, np.int64)
        kr = np.full(200, 7, np.int64)
    elif name == "extremes":
        special = np.array([i64.min, i64.max, -1, 0, 1, i64.min + 1, i64.max - 1], np.int64)
        kl = np.concatenate([special, rng.integers(i64.min, i64.max, 500, dtype=np.int64, endpoint=True)])
        kr = np.concatenate([special[::-1], kl[rng.integers(0, kl.size, 300)],
                             rng.integers(i64.min, i64.max, 200, dtype=np.int64, endpoint=True)])
        kl = kl[rng.permutation(kl.size)]
        kr = kr[rng.permutation(kr.size)]
    elif name == "int32_negative":
        kl = rng.integers(-1000, 1000, 3000, dtype=np.int64).astype(np.int32)
        kr = rng.integers(-1000, 1000, 2000, dtype=np.int64).astype(np.int32)
        return kl, _payload(kl.size), kr, _payload(kr.size), np.int32
    elif name == "int32_extremes":
        i32 = np.iinfo(np.int32)
        special = np.array([i32.min, i32.max, -1, 0, 1], np.int32)
        kl = np.concatenate([special, rng.integers(i32.min, i32.max, 400, dtype=np.int64).astype(np.int32)])
        kr = np.concatenate([special, kl[rng.integers(0, kl.size, 300)]])
        return kl, _payload(kl.size), kr, _payload(kr.size), np.int32
    else:
        raise KeyError(name)
    return kl, _payload(kl.size), kr, _payload(kr.size), np.int64


def config_inputs(name: str, seed: int | None = None, scale: float = 1.0):
    """Inputs of a named workload; ``scale`` < 1 shrinks the row counts."""
    spec = CONFIGS[name]
    seed = spec.seed if seed is None else seed
    nl = max(0, int(round(spec.n_left * scale)))
    nr = max(0, int(round(spec.n_right * scale)))
    kd = np.dtype(spec.key_dtype)
    if spec.kind == "uniform":
        kr_range = max(1, int(round(spec.key_range * scale)))
        return uniform_tables(nl, nr, kr_range, seed, kd)
    if spec.kind == "match":
        return match_fraction_tables(nl, nr, spec.frac, seed, kd)
    if spec.kind == "zipf":
        return zipf_tables(nl, nr, spec.zipf_s, spec.zipf_support, seed, kd)
    raise ValueError(spec.kind)


@dataclass(frozen=True)
class BatchMerge:
    """One merge of a batch: its index, sizes and key type."""
    index: int
    n_left: int
    n_right: int
    key_dtype: str


def batch_specs(count: int, seed: int = 0, lo: float = 1e3, hi: float = 4e6):
    """Sizes of a batch of merges: n_left and n_right independently
    log-uniform in [lo, hi] (rounded), key type int32 or int64 with
    probability 1/2 each; drawn merge by merge in that order."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nl = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        nr = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        kd = "int32" if rng.random() < 0.5 else "int64"
        out.append(BatchMerge(i, nl, nr, kd))
    return out


def batch_tables(spec: BatchMerge, frac: float = 0.3, seed: int = 0):
    """Tables of one batch merge: match_fraction_tables with the merge's
    sizes and key type, seeded by (seed, index)."""
    return match_fraction_tables(spec.n_left, spec.n_right, frac,
                                 seed=np.random.SeedSequence([seed, spec.index]),
                                 key_dtype=np.dtype(spec.key_dtype))
