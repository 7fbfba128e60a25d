"""Seeded synthetic inputs for the merge workloads.

This module only draws keys and payloads; it contains none of the method's
arithmetic (no hashing, partitioning or joining).  Both the CPU oracle and the
GPU path consume exactly the arrays produced here, so the two sides see
identical bytes.

The paper's cuDF-merge benchmark script is not part of the paper; only its
shape is printed: a chunk of 1E8 rows per worker, shuffle enabled, a "fraction
match" of 0.3, and 3.2 GB per worker (Section V-B, cuDF Merge, and the caption
of the RI2 cuDF figure), i.e. 16 bytes per row per table = one int64 key plus
one int64 payload.  The generators below reproduce that shape; see
``match_fraction_tables`` for how "fraction match" is read.
"""

from .merge_inputs import (  # noqa: F401
    CONFIGS,
    BatchMerge,
    WorkloadSpec,
    batch_specs,
    batch_tables,
    config_inputs,
    match_fraction_tables,
    uniform_tables,
    zipf_tables,
    edge_tables,
)
