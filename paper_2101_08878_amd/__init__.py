"""libmdx: one Dask worker's cuDF-merge work (hash partition + hash join) on
MI355X, behind a C ABI (include/mdx.h).  This package holds the HIP sources
(csrc/), the build script and the thin Python binding."""

from ._lib import (  # noqa: F401
    ABI_FUNCTIONS,
    KernelTrace,
    TRACEABLE_KERNELS,
    MDX_DEV_BAD_PARTITIONING,
    MDX_DEV_OUTPUT_OVERFLOW,
    MDX_ERR_HIP,
    MDX_ERR_INVALID,
    MDX_ERR_WORKSPACE,
    MDX_KEY_I32,
    MDX_KEY_I64,
    MDX_MAX_P,
    MDX_OK,
    LIB_PATH,
    MdxError,
    Table,
    abi_version,
    last_error,
    mdx_hash_partition,
    mdx_hash_partition_workspace_bytes,
    mdx_join_build,
    mdx_join_probe,
    mdx_join_probe_workspace_bytes,
    mdx_join_table_bytes,
    mdx_merge,
    mdx_merge_workspace_bytes,
    merge,
    status_string,
)
