"""Write the oracle-derived regression fixtures in tests/golden/.

Calls only the oracle (oracle/) and the seeded generators.  These values are
regression pins: they prove the oracle has not changed, not that it is right
(the independent pins live in tests/test_oracle_pins.py).

    python tests/golden/make_golden.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1
KEYS = [0, 1, 2, 3, 42, 199999, -1, I64_MAX, I64_MIN, 12345678901234, -987654321]
PS = [1, 3, 4, 8, 16, 32, 1000]


def write_fmix64():
    path = os.path.join(HERE, "fmix64_regression.txt")
    with open(path, "w") as f:
        f.write("# oracle fmix64 and fmix64 mod P; written by tests/golden/make_golden.py\n")
        f.write("# key fmix64_hex " + " ".join(f"mod{p}" for p in PS) + "\n")
        for k in KEYS:
            h = oracle.fmix64(k & 0xFFFFFFFFFFFFFFFF)
            f.write(f"{k} {h:#018x} " + " ".join(str(oracle.partition_of(k, p)) for p in PS) + "\n")


def write_paper_left_counts():
    # The left table of the 1E8-row workload is a permutation of [0, 1E8), so
    # its per-destination counts do not depend on the seed.
    n, P = 100_000_000, 32
    keys = np.arange(n, dtype=np.int64)
    _, _, off = oracle.hash_partition(keys, keys, P)
    cnt = np.diff(off)
    path = os.path.join(HERE, "paper_left_partition_counts_p32.txt")
    with open(path, "w") as f:
        f.write("# rows per destination p=0..31 of the key set [0, 1E8) under fmix64 mod 32;\n")
        f.write("# written by tests/golden/make_golden.py (oracle.hash_partition)\n")
        f.write(" ".join(str(int(c)) for c in cnt) + "\n")


if __name__ == "__main__":
    write_fmix64()
    write_paper_left_counts()
    print("ok")
