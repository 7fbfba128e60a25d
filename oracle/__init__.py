"""Python access to the C oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The GPU library and its binding
never import it.

All arrays are numpy; keys int64 or int32, payloads int64.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    i32, i64, u64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
    lib.oracle_fmix64.restype = u64
    lib.oracle_fmix64.argtypes = [u64]
    lib.oracle_partition_of.restype = i32
    lib.oracle_partition_of.argtypes = [i64, i32]
    lib.oracle_hash_partition.restype = i32
    lib.oracle_hash_partition.argtypes = [vp, i32, vp, i64, i32, vp, vp, vp]
    lib.oracle_join.restype = i64
    lib.oracle_join.argtypes = [vp, vp, i64, vp, vp, i64, i32, vp, vp, vp, i64, i32, vp]
    lib.oracle_match_counts.restype = i32
    lib.oracle_match_counts.argtypes = [vp, i64, vp, i64, i32, vp]
    lib.oracle_merge_threads.restype = i64
    lib.oracle_merge_threads.argtypes = [vp, vp, i64, vp, vp, i64, i32, i32, i32, vp, vp, vp,
                                         vp, vp, vp, vp, vp, vp, i64, vp]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def _keys(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype not in (np.int32, np.int64):
        raise TypeError(f"keys must be int32 or int64, got {a.dtype}")
    return a


def fmix64(x: int) -> int:
    """MurmurHash3's 64-bit finalizer of one uint64."""
    return int(_load().oracle_fmix64(ctypes.c_uint64(int(x) & 0xFFFFFFFFFFFFFFFF)))


def partition_of(key: int, P: int) -> int:
    """Destination of one key: fmix64(key) mod P."""
    return int(_load().oracle_partition_of(int(key), int(P)))


def hash_partition(keys, payload, P: int):
    """Stable counting sort of the rows by fmix64(key) mod P.

    Returns (keys_out, payload_out, off) with off of length P+1.
    """
    keys = _keys(keys)
    payload = np.ascontiguousarray(payload, dtype=np.int64)
    n = keys.size
    assert payload.size == n
    ko = np.empty_like(keys)
    vo = np.empty(n, np.int64)
    off = np.empty(P + 1, np.int64)
    rc = _load().oracle_hash_partition(_ptr(keys), keys.dtype.itemsize, _ptr(payload), n, P,
                                       _ptr(ko), _ptr(vo), _ptr(off))
    if rc != 0:
        raise ValueError("oracle_hash_partition: bad arguments")
    return ko, vo, off


def join(lkeys, lpay, rkeys, rpay, P: int | None = None, materialize: bool = True,
         cap: int | None = None):
    """Inner equi-join by sort-merge.

    Returns dict(total=|J|, key, lpay, rpay [canonical (lpay, rpay, key) order,
    only if materialized and |J| <= cap], per_part [if P given]).
    """
    lk, rk = _keys(lkeys), _keys(rkeys)
    if lk.dtype != rk.dtype:
        raise TypeError("left and right keys must have the same dtype")
    lv = np.ascontiguousarray(lpay, dtype=np.int64)
    rv = np.ascontiguousarray(rpay, dtype=np.int64)
    lib = _load()
    per = np.zeros(P, np.int64) if P else None
    total = lib.oracle_join(_ptr(lk), _ptr(lv), lk.size, _ptr(rk), _ptr(rv), rk.size,
                            lk.dtype.itemsize, None, None, None, 0,
                            int(P or 0), _ptr(per) if per is not None else None)
    if total < 0:
        raise ValueError("oracle_join failed")
    res = {"total": int(total)}
    if per is not None:
        res["per_part"] = per
    if materialize and (cap is None or total <= cap):
        ok = np.empty(total, np.int64)
        ol = np.empty(total, np.int64)
        orr = np.empty(total, np.int64)
        t2 = lib.oracle_join(_ptr(lk), _ptr(lv), lk.size, _ptr(rk), _ptr(rv), rk.size,
                             lk.dtype.itemsize, _ptr(ok), _ptr(ol), _ptr(orr), total, 0, None)
        assert t2 == total
        res.update(key=ok, lpay=ol, rpay=orr)
    return res


def match_counts(lkeys, rkeys) -> np.ndarray:
    """For every right row: how many left rows share its key."""
    lk, rk = _keys(lkeys), _keys(rkeys)
    out = np.empty(rk.size, np.int64)
    rc = _load().oracle_match_counts(_ptr(lk), lk.size, _ptr(rk), rk.size, lk.dtype.itemsize,
                                     _ptr(out))
    if rc != 0:
        raise ValueError("oracle_match_counts failed")
    return out


def merge_threads(lkeys, lpay, rkeys, rpay, P: int, threads: int, cap: int | None = None):
    """Both partitions and the per-destination join, over `threads` host
    threads (the CPU baseline's all-cores leg).

    Returns dict(left=(keys, payload, off), right=(...), out_off[P+1],
    total, and key/lpay/rpay in the join walk's order when |J| <= cap).
    """
    lk, rk = _keys(lkeys), _keys(rkeys)
    if lk.dtype != rk.dtype:
        raise TypeError("left and right keys must have the same dtype")
    lv = np.ascontiguousarray(lpay, dtype=np.int64)
    rv = np.ascontiguousarray(rpay, dtype=np.int64)
    nl, nr = lk.size, rk.size
    lko, rko = np.empty_like(lk), np.empty_like(rk)
    lvo, rvo = np.empty(nl, np.int64), np.empty(nr, np.int64)
    loff, roff, out_off = (np.empty(P + 1, np.int64) for _ in range(3))
    cap = nr if cap is None else int(cap)
    ok, ol, orr = (np.empty(max(cap, 1), np.int64) for _ in range(3))
    total = _load().oracle_merge_threads(
        _ptr(lk), _ptr(lv), nl, _ptr(rk), _ptr(rv), nr, lk.dtype.itemsize, int(P), int(threads),
        _ptr(lko), _ptr(lvo), _ptr(loff), _ptr(rko), _ptr(rvo), _ptr(roff),
        _ptr(ok), _ptr(ol), _ptr(orr), cap, _ptr(out_off))
    if total < 0:
        raise ValueError("oracle_merge_threads failed")
    res = {"left": (lko, lvo, loff), "right": (rko, rvo, roff), "out_off": out_off,
           "total": int(total)}
    if total <= cap:
        res.update(key=ok[:total], lpay=ol[:total], rpay=orr[:total])
    return res


def transpose_sum(x) -> np.ndarray:
    """y = x + x^T for a square float64 matrix.

    arXiv 2101.08878, Section V-B ("Sum of cuPy Array and its Transpose"):
    the benchmark evaluates y = x + x.T on a chunked cuPy array (16K x 16K,
    4K chunks on RI2).  The plain definition: every element y[i, j] is the
    IEEE-754 double sum (round to nearest, ties to even) of x[i, j] and
    x[j, i]; numpy's elementwise add of x and its transposed view computes
    exactly that.  The paper does not state the element type; cuPy's random
    arrays are float64, which is the reading taken here.
    """
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != 2 or x.shape[0] != x.shape[1]:
        raise ValueError("transpose_sum needs a square matrix")
    return x + x.T
