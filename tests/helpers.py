"""Test-side checks shared by the oracle pins and the GPU parity tests.

Pure numpy.  Nothing here is imported by the GPU library or by the oracle.
"""

from __future__ import annotations

import numpy as np

M64 = (1 << 64) - 1


def canonical(key, lpay, rpay):
    """Sort join rows by (left payload, right payload, key)."""
    key = np.asarray(key, np.int64)
    lpay = np.asarray(lpay, np.int64)
    rpay = np.asarray(rpay, np.int64)
    order = np.lexsort((key, rpay, lpay))
    return key[order], lpay[order], rpay[order]


def brute_force_join(kl, vl, kr, vr):
    """Nested loop over all (i, j) pairs; tiny inputs only."""
    rows = []
    for i in range(len(kl)):
        for j in range(len(kr)):
            if int(kl[i]) == int(kr[j]):
                rows.append((int(kl[i]), int(vl[i]), int(vr[j])))
    if not rows:
        z = np.zeros(0, np.int64)
        return z, z.copy(), z.copy()
    a = np.array(rows, dtype=np.int64)
    return canonical(a[:, 0], a[:, 1], a[:, 2])


def expected_cardinality(kl, kr) -> int:
    """|J| = sum over keys of countL(k) * countR(k), in exact integers."""
    ul, cl = np.unique(np.asarray(kl, np.int64), return_counts=True)
    ur, cr = np.unique(np.asarray(kr, np.int64), return_counts=True)
    common, il, ir = np.intersect1d(ul, ur, assume_unique=True, return_indices=True)
    return int(np.sum(cl[il].astype(object) * cr[ir].astype(object))) if common.size else 0


def check_partition_invariants(keys_in, keys_out, pay_out, off, P, part_of_keys):
    """Invariants of a stable partition whose input payload is the row index.

    ``part_of_keys(keys) -> destinations`` must compute fmix64(key) mod P.
    """
    n = len(keys_in)
    off = np.asarray(off, np.int64)
    assert off.shape == (P + 1,)
    assert off[0] == 0 and off[-1] == n
    assert np.all(np.diff(off) >= 0)
    pay_out = np.asarray(pay_out, np.int64)
    # every row lands exactly once
    assert np.array_equal(np.sort(pay_out), np.arange(n, dtype=np.int64))
    # keys travel with their payload
    assert np.array_equal(np.asarray(keys_out), np.asarray(keys_in)[pay_out])
    dest = np.repeat(np.arange(P), np.diff(off))
    assert np.array_equal(part_of_keys(np.asarray(keys_out)), dest)
    # stability: inside a destination, original indices increase
    if n > 1:
        same = dest[1:] == dest[:-1]
        assert np.all(pay_out[1:][same] > pay_out[:-1][same])


def check_join_rows(kl, kr, key, lpay, rpay, lpay_is_index=True):
    """Every output row is a genuine match and no (l, r) pair repeats."""
    key = np.asarray(key, np.int64)
    lpay = np.asarray(lpay, np.int64)
    rpay = np.asarray(rpay, np.int64)
    if key.size == 0:
        return
    assert np.array_equal(np.asarray(kl, np.int64)[lpay], key)
    assert np.array_equal(np.asarray(kr, np.int64)[rpay], key)
    pair = lpay.astype(np.uint64) * np.uint64(len(kr) + 1) + rpay.astype(np.uint64)
    assert np.unique(pair).size == pair.size


# ---- an fmix64 for numpy arrays, used only to check destinations ---------
def fmix64_np(keys) -> np.ndarray:
    x = np.asarray(keys).astype(np.int64).view(np.uint64).copy()
    with np.errstate(over="ignore"):
        x ^= x >> np.uint64(33)
        x *= np.uint64(0xFF51AFD7ED558CCD)
        x ^= x >> np.uint64(33)
        x *= np.uint64(0xC4CEB9FE1A85EC53)
        x ^= x >> np.uint64(33)
    return x


def part_np(keys, P) -> np.ndarray:
    return (fmix64_np(keys) % np.uint64(P)).astype(np.int64)
