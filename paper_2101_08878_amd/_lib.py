"""ctypes binding of libmdx (include/mdx.h).

Argument marshalling only: tensors are checked for device, dtype and
contiguity and their raw pointers are forwarded; every step of the hash
partition and join runs in libmdx's HIP kernels.  torch supplies device
memory (output and workspace tensors) and streams.  There is no CPU
fallback: if libmdx.so is missing, importing this module raises.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdx.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mdx.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libmdx.so not found at {LIB_PATH}; build it with `python -m paper_2101_08878_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)


MDX_OK = 0
MDX_ERR_INVALID = 1
MDX_ERR_WORKSPACE = 2
MDX_ERR_HIP = 3
MDX_BUSY = 4
MDX_KEY_I32 = 4
MDX_KEY_I64 = 8
MDX_DEV_OUTPUT_OVERFLOW = 1
MDX_DEV_BAD_PARTITIONING = 2
MDX_DEV_SCAN_TIMEOUT = 4
MDX_MAX_P = 4096
MDX_MAX_LANES = 8
MDX_NOALLOC_SCRATCH_BYTES = 16 << 20
MDX_MAX_SLOTS = 32
MDX_MAX_TRANSPOSE_N = 1 << 17

_i32, _i64, _sz, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p


class mdx_table(ctypes.Structure):
    _fields_ = [
        ("abi_version", _i32), ("P", _i32), ("key_type", _i32), ("reserved", _i32),
        ("n", _i64), ("d_mem", _vp), ("bytes", _sz),
        ("d_offsets", _vp), ("d_flags", _vp), ("d_bump", _vp),
        ("d_slots", _vp), ("d_gstart", _vp), ("d_grouped", _vp),
    ]


class mdx_merge_desc(ctypes.Structure):
    _fields_ = [
        ("d_left_keys", _vp), ("d_left_payload", _vp), ("n_left", _i64),
        ("d_right_keys", _vp), ("d_right_payload", _vp), ("n_right", _i64),
        ("key_type", _i32), ("P", _i32),
        ("d_out_key", _vp), ("d_out_lpay", _vp), ("d_out_rpay", _vp), ("out_capacity", _i64),
        ("d_out_offsets", _vp), ("d_status", _vp),
    ]


class mdx_batch_tuning(ctypes.Structure):
    _fields_ = [("fill", ctypes.c_float), ("fanout", _i32), ("part_rows", _i32), ("reserved", _i32)]


class mdx_probe_desc(ctypes.Structure):
    _fields_ = [
        ("d_keys", _vp), ("d_payload", _vp), ("n", _i64),
        ("d_out_key", _vp), ("d_out_lpay", _vp), ("d_out_rpay", _vp), ("out_capacity", _i64),
        ("d_out_offsets", _vp), ("d_status", _vp),
    ]


def _sig(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_abi_version = _sig("mdx_abi_version", _i32)
_status_string = _sig("mdx_status_string", ctypes.c_char_p, _i32)
_last_error = _sig("mdx_last_error", ctypes.c_char_p)
_part_ws = _sig("mdx_hash_partition_workspace_bytes", _i32, _i64, _i32, _i32, ctypes.POINTER(_sz))
_part = _sig("mdx_hash_partition", _i32, _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp)
_part_noalloc = _sig("mdx_hash_partition_noalloc", _i32, _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp,
                     _vp)
_table_bytes = _sig("mdx_join_table_bytes", _i32, _i64, _i32, _i32, ctypes.POINTER(_sz))
_build = _sig("mdx_join_build", _i32, _vp, _vp, _vp, _i64, _i32, _i32, _vp, _sz,
              ctypes.POINTER(mdx_table), _vp, _vp)
_probe_ws = _sig("mdx_join_probe_workspace_bytes", _i32, _i64, _i32, _i32, ctypes.POINTER(_sz))
_probe = _sig("mdx_join_probe", _i32, ctypes.POINTER(mdx_table), _vp, _vp, _vp, _i64, _vp, _sz,
              _vp, _vp, _vp, _i64, _vp, _vp, _vp)
_count_ws = _sig("mdx_join_count_workspace_bytes", _i32, _i64, _i64, _i32, _i32, ctypes.POINTER(_sz))
_count = _sig("mdx_join_count", _i32, _vp, _vp, _i64, _vp, _vp, _i64, _i32, _i32, _vp, _sz, _vp, _vp,
              _vp)
_merge_ws = _sig("mdx_merge_workspace_bytes", _i32, _i64, _i64, _i32, _i32, ctypes.POINTER(_sz))
_merge = _sig("mdx_merge", _i32, _vp, _vp, _i64, _vp, _vp, _i64, _i32, _i32, _vp, _sz,
              _vp, _vp, _vp, _i64, _vp, _vp, _vp)

_batch_ws = _sig("mdx_merge_batch_workspace_bytes", _i32, _i32, ctypes.POINTER(mdx_merge_desc), _i32,
                 ctypes.POINTER(_sz))
_batch = _sig("mdx_merge_batch", _i32, _i32, ctypes.POINTER(mdx_merge_desc), _i32, _vp, _sz, _vp)

_fb_ws = _sig("mdx_batch_workspace_bytes", _i32, _i32, ctypes.POINTER(mdx_merge_desc),
               ctypes.POINTER(mdx_batch_tuning), ctypes.POINTER(_sz), ctypes.POINTER(_sz))
_fb_create = _sig("mdx_batch_create", _i32, _i32, ctypes.POINTER(mdx_merge_desc),
                  ctypes.POINTER(mdx_batch_tuning), _vp, _sz, ctypes.POINTER(_vp))
_fb_info = _sig("mdx_batch_info", _i32, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32))
_fb_run = _sig("mdx_batch_run", _i32, _vp, _vp)
_fb_destroy = _sig("mdx_batch_destroy", _i32, _vp)

_srv_ws = _sig("mdx_server_workspace_bytes", _i32, _i32, _i64, _i64, _i32, ctypes.POINTER(_sz))
_srv_create = _sig("mdx_server_create", _i32, _i32, _i64, _i64, _i32, _sz, _vp, _sz,
                   ctypes.POINTER(_vp))
_srv_submit = _sig("mdx_server_submit", _i32, _vp, ctypes.POINTER(mdx_merge_desc), _i64, _vp,
                   ctypes.POINTER(_i32))
_srv_submit_probe = _sig("mdx_server_submit_probe", _i32, _vp, ctypes.POINTER(mdx_table),
                         ctypes.POINTER(mdx_probe_desc), _i64, _vp, ctypes.POINTER(_i32))
_srv_poll = _sig("mdx_server_poll", _i32, _vp, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_i32))
_srv_stats = _sig("mdx_server_stats", _i32, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_sz))
_srv_destroy = _sig("mdx_server_destroy", _i32, _vp)

_tsum = _sig("mdx_transpose_sum", _i32, _vp, _vp, _i64, _vp)

_trace = _sig("mdx_trace_kernel", _i32, ctypes.c_char_p, _vp, _vp, _i32, ctypes.POINTER(_i32))

ABI_FUNCTIONS = [
    "mdx_abi_version", "mdx_status_string", "mdx_last_error",
    "mdx_hash_partition_workspace_bytes", "mdx_hash_partition", "mdx_hash_partition_noalloc",
    "mdx_join_table_bytes", "mdx_join_build",
    "mdx_join_probe_workspace_bytes", "mdx_join_probe",
    "mdx_join_count_workspace_bytes", "mdx_join_count",
    "mdx_merge_workspace_bytes", "mdx_merge",
    "mdx_merge_batch_workspace_bytes", "mdx_merge_batch",
    "mdx_batch_workspace_bytes", "mdx_batch_create", "mdx_batch_info", "mdx_batch_run",
    "mdx_batch_destroy",
    "mdx_server_workspace_bytes", "mdx_server_create", "mdx_server_submit",
    "mdx_server_submit_probe", "mdx_server_poll",
    "mdx_server_stats", "mdx_server_destroy",
    "mdx_transpose_sum",
    "mdx_trace_kernel",
]
TRACEABLE_KERNELS = ["part_hist", "part_scatter", "seg_hist", "seg_scatter", "rj_join", "cnt_insert",
                     "cnt_probe", "grp_count",
                     "grp_alloc", "grp_scatter",
                     "tbl_init", "tbl_insert", "probe_chain", "probe_expand", "transpose_sum"]


class MdxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_status_string(status).decode()} ({status}): {message}")
        self.status = status


def _check(status: int):
    if status != MDX_OK:
        raise MdxError(status, _last_error().decode())


def abi_version() -> int:
    return int(_abi_version())


def status_string(status: int) -> str:
    return _status_string(int(status)).decode()


def last_error() -> str:
    return _last_error().decode()


# ---- marshalling helpers -----------------------------------------------------

def _key_type(t: torch.Tensor) -> int:
    if t.dtype == torch.int64:
        return MDX_KEY_I64
    if t.dtype == torch.int32:
        return MDX_KEY_I32
    raise TypeError(f"keys must be int32 or int64, got {t.dtype}")


def _dev(t: torch.Tensor, name: str, dtype=None, n=None) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")
    return t.data_ptr() if t.numel() else 0


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _bytes(fn, *args) -> int:
    out = _sz(0)
    _check(fn(*args, ctypes.byref(out)))
    return int(out.value)


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def _handoff(stream, made):
    """Tensors allocated here (`made`: workspaces, missing outputs) come from
    the current stream's pool; when the work goes to another stream, that
    stream first waits for the current one (so it never touches memory the
    current stream's earlier work still uses) and the tensors are marked as
    used on it (so the allocator hands them out again only after that work)."""
    made = [t for t in made if t is not None]
    if stream is None or not made:
        return
    cur = torch.cuda.current_stream(made[0].device)
    if stream == cur:
        return
    stream.wait_stream(cur)
    for t in made:
        t.record_stream(stream)


# ---- hash partition ------------------------------------------------------------

def mdx_hash_partition_workspace_bytes(n: int, P: int, key_type: int = MDX_KEY_I64) -> int:
    return _bytes(_part_ws, int(n), int(P), int(key_type))


def mdx_hash_partition(keys: torch.Tensor, payload: torch.Tensor, P: int, *, keys_out=None,
                       payload_out=None, offsets=None, workspace=None, stream=None):
    """Stable partition by fmix64(key) mod P.  Returns (keys_out, payload_out,
    offsets[P+1]) as device tensors; the work is enqueued on `stream`."""
    n = keys.numel()
    kt = _key_type(keys)
    dev = keys.device
    made = []
    if keys_out is None:
        keys_out = torch.empty_like(keys)
        made.append(keys_out)
    if payload_out is None:
        payload_out = torch.empty(n, dtype=torch.int64, device=dev)
        made.append(payload_out)
    if offsets is None:
        offsets = torch.empty(P + 1, dtype=torch.int64, device=dev)
        made.append(offsets)
    if workspace is None:
        workspace = _workspace(mdx_hash_partition_workspace_bytes(n, P, kt), dev)
        made.append(workspace)
    _handoff(stream, made)
    _check(_part(_dev(keys, "keys"), _dev(payload, "payload", torch.int64, n), n, kt, int(P),
                 _dev(keys_out, "keys_out", keys.dtype, n), _dev(payload_out, "payload_out", torch.int64, n),
                 _dev(offsets, "offsets", torch.int64, P + 1), _dev(workspace, "workspace"),
                 workspace.numel() * workspace.element_size(), _stream(stream)))
    return keys_out, payload_out, offsets


def mdx_hash_partition_noalloc(keys: torch.Tensor, payload: torch.Tensor, P: int, *, keys_out,
                               payload_out, offsets, stream=None):
    """mdx_hash_partition with the library's own scratch array as its
    workspace (for callers that cannot allocate).  The outputs are the
    caller's; nothing is allocated here or in the call."""
    n = keys.numel()
    kt = _key_type(keys)
    _check(_part_noalloc(_dev(keys, "keys"), _dev(payload, "payload", torch.int64, n), n, kt, int(P),
                         _dev(keys_out, "keys_out", keys.dtype, n),
                         _dev(payload_out, "payload_out", torch.int64, n),
                         _dev(offsets, "offsets", torch.int64, P + 1), _stream(stream)))
    return keys_out, payload_out, offsets


# ---- join -------------------------------------------------------------------------

@dataclass
class Table:
    """A built table: the C struct plus the tensor that owns its memory."""
    struct: mdx_table
    memory: torch.Tensor

    @property
    def P(self) -> int:
        return int(self.struct.P)


def mdx_join_table_bytes(n_build: int, P: int, key_type: int = MDX_KEY_I64) -> int:
    return _bytes(_table_bytes, int(n_build), int(P), int(key_type))


def mdx_join_build(keys: torch.Tensor, payload: torch.Tensor, offsets: torch.Tensor, P: int, *,
                   table_memory=None, status=None, stream=None) -> Table:
    n = keys.numel()
    kt = _key_type(keys)
    need = mdx_join_table_bytes(n, P, kt)
    mem = _workspace(need, keys.device) if table_memory is None else table_memory
    _handoff(stream, [mem] if table_memory is None else [])
    t = mdx_table()
    _check(_build(_dev(keys, "keys"), _dev(payload, "payload", torch.int64, n),
                  _dev(offsets, "offsets", torch.int64, P + 1), n, int(P), kt, _dev(mem, "table_memory"),
                  mem.numel() * mem.element_size(), ctypes.byref(t),
                  _dev(status, "status", torch.int32, 1) if status is not None else None,
                  _stream(stream)))
    return Table(t, mem)


def mdx_join_probe_workspace_bytes(n_probe: int, P: int, key_type: int = MDX_KEY_I64) -> int:
    return _bytes(_probe_ws, int(n_probe), int(P), int(key_type))


def _outputs(cap: int, key_dtype, device, out):
    if out is not None:
        return out
    return (torch.empty(cap, dtype=key_dtype, device=device),
            torch.empty(cap, dtype=torch.int64, device=device),
            torch.empty(cap, dtype=torch.int64, device=device))


def mdx_join_probe(table: Table, keys: torch.Tensor, payload: torch.Tensor, offsets: torch.Tensor, *,
                   out_capacity: int, out=None, out_offsets=None, workspace=None, status=None,
                   stream=None):
    """Probe a built table.  Returns (out_key, out_lpay, out_rpay, out_offsets).
    Rows of partition p are at [out_offsets[p], out_offsets[p+1]); if
    out_offsets[P] > out_capacity the rows are not all written and
    MDX_DEV_OUTPUT_OVERFLOW is set in `status`."""
    n = keys.numel()
    P = table.P
    kt = _key_type(keys)
    dev = keys.device
    made = []
    ok, ol, orr = _outputs(out_capacity, keys.dtype, dev, out)
    if out is None:
        made += [ok, ol, orr]
    if out_offsets is None:
        out_offsets = torch.empty(P + 1, dtype=torch.int64, device=dev)
        made.append(out_offsets)
    if workspace is None:
        workspace = _workspace(mdx_join_probe_workspace_bytes(n, P, kt), dev)
        made.append(workspace)
    _handoff(stream, made)
    _check(_probe(ctypes.byref(table.struct), _dev(keys, "keys"), _dev(payload, "payload", torch.int64, n),
                  _dev(offsets, "offsets", torch.int64, P + 1), n, _dev(workspace, "workspace"),
                  workspace.numel() * workspace.element_size(),
                  _dev(ok, "out_key", keys.dtype, out_capacity), _dev(ol, "out_lpay", torch.int64, out_capacity),
                  _dev(orr, "out_rpay", torch.int64, out_capacity), int(out_capacity),
                  _dev(out_offsets, "out_offsets", torch.int64, P + 1),
                  _dev(status, "status", torch.int32, 1) if status is not None else None,
                  _stream(stream)))
    return ok, ol, orr, out_offsets


def mdx_join_count_workspace_bytes(n_build: int, n_probe: int, P: int,
                                   key_type: int = MDX_KEY_I64) -> int:
    return _bytes(_count_ws, int(n_build), int(n_probe), int(P), int(key_type))


def mdx_join_count(left_keys: torch.Tensor, left_offsets: torch.Tensor, right_keys: torch.Tensor,
                   right_offsets: torch.Tensor, P: int, *, out_offsets=None, workspace=None,
                   status=None, stream=None):
    """Per-partition output counts of the inner join of two partitioned
    tables (as mdx_join_probe's offsets), without materializing it.
    Asynchronous; returns out_offsets [P+1] (total at [P])."""
    nl, nr = left_keys.numel(), right_keys.numel()
    kt = _key_type(left_keys)
    if right_keys.dtype != left_keys.dtype:
        raise TypeError("left and right keys must have the same dtype")
    dev = left_keys.device
    made = []
    if out_offsets is None:
        out_offsets = torch.empty(P + 1, dtype=torch.int64, device=dev)
        made.append(out_offsets)
    if workspace is None:
        workspace = _workspace(mdx_join_count_workspace_bytes(nl, nr, P, kt), dev)
        made.append(workspace)
    _handoff(stream, made)
    _check(_count(_dev(left_keys, "left_keys"), _dev(left_offsets, "left_offsets", torch.int64, P + 1),
                  nl, _dev(right_keys, "right_keys"),
                  _dev(right_offsets, "right_offsets", torch.int64, P + 1), nr, int(P), kt,
                  _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(),
                  _dev(out_offsets, "out_offsets", torch.int64, P + 1),
                  _dev(status, "status", torch.int32, 1) if status is not None else None,
                  _stream(stream)))
    return out_offsets


# ---- merge ---------------------------------------------------------------------------

def mdx_merge_workspace_bytes(n_left: int, n_right: int, P: int, key_type: int = MDX_KEY_I64) -> int:
    return _bytes(_merge_ws, int(n_left), int(n_right), int(P), int(key_type))


def mdx_merge(left_keys: torch.Tensor, left_payload: torch.Tensor, right_keys: torch.Tensor,
              right_payload: torch.Tensor, P: int, *, out_capacity: int, out=None, out_offsets=None,
              workspace=None, status=None, stream=None):
    """Partition both tables into P destinations and join every partition.
    Asynchronous; returns (out_key, out_lpay, out_rpay, out_offsets)."""
    nl, nr = left_keys.numel(), right_keys.numel()
    kt = _key_type(left_keys)
    if right_keys.dtype != left_keys.dtype:
        raise TypeError("left and right keys must have the same dtype")
    dev = left_keys.device
    made = []
    ok, ol, orr = _outputs(out_capacity, left_keys.dtype, dev, out)
    if out is None:
        made += [ok, ol, orr]
    if out_offsets is None:
        out_offsets = torch.empty(P + 1, dtype=torch.int64, device=dev)
        made.append(out_offsets)
    if workspace is None:
        workspace = _workspace(mdx_merge_workspace_bytes(nl, nr, P, kt), dev)
        made.append(workspace)
    _handoff(stream, made)
    _check(_merge(_dev(left_keys, "left_keys"), _dev(left_payload, "left_payload", torch.int64, nl), nl,
                  _dev(right_keys, "right_keys"), _dev(right_payload, "right_payload", torch.int64, nr), nr,
                  kt, int(P), _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(),
                  _dev(ok, "out_key", left_keys.dtype, out_capacity),
                  _dev(ol, "out_lpay", torch.int64, out_capacity),
                  _dev(orr, "out_rpay", torch.int64, out_capacity), int(out_capacity),
                  _dev(out_offsets, "out_offsets", torch.int64, P + 1),
                  _dev(status, "status", torch.int32, 1) if status is not None else None,
                  _stream(stream)))
    return ok, ol, orr, out_offsets


def merge(left_keys, left_payload, right_keys, right_payload, P: int, *, capacity_hint=None,
          stream=None):
    """Synchronous convenience: mdx_merge, sized by a second call when the
    first output capacity is too small.  Returns (key, lpay, rpay,
    out_offsets) trimmed to the result."""
    cap = int(capacity_hint if capacity_hint is not None else max(right_keys.numel(), 1))
    for _ in range(2):
        status = torch.zeros(1, dtype=torch.int32, device=left_keys.device)
        ok, ol, orr, off = mdx_merge(left_keys, left_payload, right_keys, right_payload, P,
                                     out_capacity=cap, status=status, stream=stream)
        torch.cuda.synchronize(left_keys.device)
        total = int(off[-1].item())
        st = int(status.item())
        if st & (MDX_DEV_BAD_PARTITIONING | MDX_DEV_SCAN_TIMEOUT):
            raise MdxError(MDX_ERR_INVALID, f"device reported status {st}")
        if total <= cap and not (st & MDX_DEV_OUTPUT_OVERFLOW):
            return ok[:total], ol[:total], orr[:total], off
        cap = total
    raise MdxError(MDX_ERR_INVALID, "output capacity retry failed")


# ---- batched merges ---------------------------------------------------------------------

@dataclass
class MergeJob:
    """One merge of a batch: mdx_merge's inputs and (optionally) outputs."""
    left_keys: torch.Tensor
    left_payload: torch.Tensor
    right_keys: torch.Tensor
    right_payload: torch.Tensor
    P: int
    out_capacity: int
    out: tuple | None = None
    out_offsets: torch.Tensor | None = None
    status: torch.Tensor | None = None


@dataclass
class ProbeJob:
    """One probe of a device-resident table (Server.submit_probe)."""
    table: "Table"
    keys: torch.Tensor
    payload: torch.Tensor
    out_capacity: int
    out: tuple | None = None
    out_offsets: torch.Tensor | None = None
    status: torch.Tensor | None = None


def _batch_descs(jobs, with_pointers: bool):
    descs = (mdx_merge_desc * max(len(jobs), 1))()
    for i, j in enumerate(jobs):
        d = descs[i]
        if j.right_keys.dtype != j.left_keys.dtype:
            raise TypeError(f"merge {i}: left and right keys must have the same dtype")
        d.n_left, d.n_right = j.left_keys.numel(), j.right_keys.numel()
        d.key_type, d.P, d.out_capacity = _key_type(j.left_keys), int(j.P), int(j.out_capacity)
        if with_pointers:
            nl, nr, cap, kd = d.n_left, d.n_right, d.out_capacity, j.left_keys.dtype
            d.d_left_keys = _dev(j.left_keys, "left_keys")
            d.d_left_payload = _dev(j.left_payload, "left_payload", torch.int64, nl)
            d.d_right_keys = _dev(j.right_keys, "right_keys")
            d.d_right_payload = _dev(j.right_payload, "right_payload", torch.int64, nr)
            d.d_out_key = _dev(j.out[0], "out_key", kd, cap)
            d.d_out_lpay = _dev(j.out[1], "out_lpay", torch.int64, cap)
            d.d_out_rpay = _dev(j.out[2], "out_rpay", torch.int64, cap)
            d.d_out_offsets = _dev(j.out_offsets, "out_offsets", torch.int64, j.P + 1)
            d.d_status = _dev(j.status, "status", torch.int32, 1) if j.status is not None else None
    return descs


def mdx_merge_batch_workspace_bytes(jobs, lanes: int) -> int:
    """Workspace bytes of mdx_merge_batch for these jobs (sizes only)."""
    return _bytes(_batch_ws, len(jobs), _batch_descs(jobs, False), int(lanes))


def mdx_merge_batch(jobs, *, lanes: int = 4, workspace=None, stream=None):
    """Run every MergeJob as mdx_merge would, on up to `lanes` concurrent
    lanes.  Missing outputs are allocated here.  Asynchronous; returns the
    jobs with their outputs filled in."""
    made = []
    for j in jobs:
        dev = j.left_keys.device
        if j.out is None:
            j.out = _outputs(j.out_capacity, j.left_keys.dtype, dev, None)
            made += list(j.out)
        if j.out_offsets is None:
            j.out_offsets = torch.empty(j.P + 1, dtype=torch.int64, device=dev)
            made.append(j.out_offsets)
    if workspace is None:
        need = mdx_merge_batch_workspace_bytes(jobs, lanes)
        dev = jobs[0].left_keys.device if jobs else torch.device("cuda")
        workspace = _workspace(need, dev)
        made.append(workspace)
    _handoff(stream, made)
    descs = _batch_descs(jobs, True)
    _check(_batch(len(jobs), descs, int(lanes), _dev(workspace, "workspace"),
                  workspace.numel() * workspace.element_size(), _stream(stream)))
    return jobs


# ---- fused batches ------------------------------------------------------------------------

def _tunings(jobs, tuning):
    """ctypes array of per-merge tuning, or None for the library defaults.
    `tuning`: None, "table" (paper_2101_08878_amd/tuning.json by key width
    and size), one dict for every merge, or a list of dicts (keys fill,
    fanout, part_rows; missing keys mean the default)."""
    if tuning is None or not jobs:
        return None
    if tuning == "table":
        from .autotune import lookup
        per = [lookup(j.left_keys.element_size(), max(j.left_keys.numel(), j.right_keys.numel()))
               for j in jobs]
    elif isinstance(tuning, dict):
        per = [tuning] * len(jobs)
    else:
        per = list(tuning)
        if len(per) != len(jobs):
            raise ValueError("one tuning entry per merge")
    arr = (mdx_batch_tuning * len(jobs))()
    for i, t in enumerate(per):
        arr[i].fill = float(t.get("fill", 0.0))
        arr[i].fanout = int(t.get("fanout", 0))
        arr[i].part_rows = int(t.get("part_rows", 0))
    return arr


def mdx_batch_workspace_bytes(jobs, tuning=None):
    """(least, one-wave) workspace bytes of a fused batch of these jobs."""
    lo, hi = _sz(0), _sz(0)
    _check(_fb_ws(len(jobs), _batch_descs(jobs, False), _tunings(jobs, tuning), ctypes.byref(lo),
                  ctypes.byref(hi)))
    return int(lo.value), int(hi.value)


class FusedBatch:
    """A fused batch (mdx_batch_*): every merge's steps in one launch per
    step.  Plans the jobs once (outputs missing from a job and the workspace
    are allocated here); run() enqueues the batch and may be called again or
    captured into a HIP graph.  The object keeps the jobs' tensors and the
    workspace alive; close() (or garbage collection) frees the plan after
    the caller has synchronized with every run."""

    def __init__(self, jobs, *, tuning=None, workspace=None, workspace_bytes: int | None = None):
        self.jobs = list(jobs)
        made = []
        for j in self.jobs:
            dev = j.left_keys.device
            if j.out is None:
                j.out = _outputs(j.out_capacity, j.left_keys.dtype, dev, None)
                made += list(j.out)
            if j.out_offsets is None:
                j.out_offsets = torch.empty(j.P + 1, dtype=torch.int64, device=dev)
                made.append(j.out_offsets)
        self._tuning = _tunings(self.jobs, tuning)
        lo, hi = mdx_batch_workspace_bytes(self.jobs, tuning)
        if workspace is None:
            need = hi if workspace_bytes is None else max(lo, min(hi, int(workspace_bytes)))
            dev = self.jobs[0].left_keys.device if self.jobs else torch.device("cuda")
            workspace = _workspace(need, dev)
            made.append(workspace)
        self.workspace = workspace
        self._made = made
        self._handed = False
        descs = _batch_descs(self.jobs, True)
        h = _vp()
        _check(_fb_create(len(self.jobs), descs, self._tuning, _dev(workspace, "workspace"),
                          workspace.numel() * workspace.element_size(), ctypes.byref(h)))
        self._h = h

    def info(self):
        """(waves, kernel launches) of one run."""
        w, n = _i32(0), _i32(0)
        _check(_fb_info(self._h, ctypes.byref(w), ctypes.byref(n)))
        return int(w.value), int(n.value)

    def run(self, stream=None):
        if self._h is None:
            raise MdxError(MDX_ERR_INVALID, "batch is closed")
        if not self._handed:
            _handoff(stream, self._made)
            self._handed = True
        _check(_fb_run(self._h, _stream(stream)))
        return self.jobs

    def close(self):
        if getattr(self, "_h", None) is not None:
            _check(_fb_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving ------------------------------------------------------------------------------

def mdx_server_workspace_bytes(slots: int, max_left: int, max_right: int, max_P: int) -> int:
    return _bytes(_srv_ws, int(slots), int(max_left), int(max_right), int(max_P))


class Server:
    """Merge requests admitted as slots and memory free up (mdx_server_*).

    submit() returns the slot a MergeJob went to, or None when no slot or
    budget is free (nothing enqueued); poll() returns the tags of finished
    merges.  The server keeps each job (and so its buffers) until it is
    polled.  One host thread at a time."""

    def __init__(self, slots: int, max_left: int, max_right: int, max_P: int,
                 budget_bytes: int, device=None):
        device = torch.device("cuda") if device is None else device
        need = mdx_server_workspace_bytes(slots, max_left, max_right, max_P)
        self.workspace = _workspace(need, device)
        h = _vp()
        _check(_srv_create(int(slots), int(max_left), int(max_right), int(max_P), int(budget_bytes),
                           _dev(self.workspace, "workspace"), self.workspace.numel(), ctypes.byref(h)))
        self._h = h
        self._tags = (_i64 * int(slots))()
        self._jobs = {}

    @staticmethod
    def _ready(ready):
        """The event a request waits for before reading its inputs: by
        default one recorded now on the current stream, which orders the
        inputs written there and the outputs allocated there before the
        slot's stream; 0 waits for nothing (inputs and outputs already
        complete).  Returns (handle, event kept alive until submitted)."""
        if ready is not None:
            return ready, None
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        return ev.cuda_event, ev

    def submit(self, job: MergeJob, tag: int, ready=None):
        if self._h is None:
            raise MdxError(MDX_ERR_INVALID, "server is closed")
        dev = job.left_keys.device
        if job.out is None:
            job.out = _outputs(job.out_capacity, job.left_keys.dtype, dev, None)
        if job.out_offsets is None:
            job.out_offsets = torch.empty(job.P + 1, dtype=torch.int64, device=dev)
        desc = _batch_descs([job], True)
        slot = _i32(-1)
        handle, _keep = self._ready(ready)
        st = _srv_submit(self._h, desc, int(tag), handle, ctypes.byref(slot))
        if st == MDX_BUSY:
            return None
        _check(st)
        self._jobs[int(tag)] = job
        return slot.value

    def submit_probe(self, job: "ProbeJob", tag: int, ready=None):
        """Probe job.table (built once with mdx_join_build, kept on the
        device) with job's rows in a free slot; None when no slot or budget
        is free (nothing enqueued)."""
        if self._h is None:
            raise MdxError(MDX_ERR_INVALID, "server is closed")
        t = job.table
        dev = job.keys.device
        if job.out is None:
            job.out = _outputs(job.out_capacity, job.keys.dtype, dev, None)
        if job.out_offsets is None:
            job.out_offsets = torch.empty(t.P + 1, dtype=torch.int64, device=dev)
        n, cap = job.keys.numel(), int(job.out_capacity)
        d = mdx_probe_desc()
        d.d_keys = _dev(job.keys, "keys")
        d.d_payload = _dev(job.payload, "payload", torch.int64, n)
        d.n = n
        d.d_out_key = _dev(job.out[0], "out_key", job.keys.dtype, cap)
        d.d_out_lpay = _dev(job.out[1], "out_lpay", torch.int64, cap)
        d.d_out_rpay = _dev(job.out[2], "out_rpay", torch.int64, cap)
        d.out_capacity = cap
        d.d_out_offsets = _dev(job.out_offsets, "out_offsets", torch.int64, t.P + 1)
        d.d_status = _dev(job.status, "status", torch.int32, 1) if job.status is not None else None
        slot = _i32(-1)
        handle, _keep = self._ready(ready)
        st = _srv_submit_probe(self._h, ctypes.byref(t.struct), ctypes.byref(d), int(tag), handle,
                               ctypes.byref(slot))
        if st == MDX_BUSY:
            return None
        _check(st)
        self._jobs[int(tag)] = job
        return slot.value

    def poll(self):
        n = _i32(0)
        _check(_srv_poll(self._h, self._tags, len(self._tags), ctypes.byref(n)))
        done = [self._tags[i] for i in range(n.value)]
        for t in done:
            self._jobs.pop(t, None)
        return done

    def stats(self):
        b, nbytes = _i32(0), _sz(0)
        _check(_srv_stats(self._h, ctypes.byref(b), ctypes.byref(nbytes)))
        return b.value, nbytes.value

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            _check(_srv_destroy(h))
            self._jobs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- transpose sum ----------------------------------------------------------------------

def mdx_transpose_sum(x: torch.Tensor, *, out=None, stream=None) -> torch.Tensor:
    """y = x + x^T for a square float64 matrix (out may be x).  Asynchronous."""
    if x.dim() != 2 or x.shape[0] != x.shape[1]:
        raise ValueError("x must be a square matrix")
    n = x.shape[0]
    out = torch.empty_like(x) if out is None else out
    if out.shape != x.shape:
        raise ValueError("out must have the shape of x")
    _check(_tsum(_dev(x, "x", torch.float64), _dev(out, "out", torch.float64), n, _stream(stream)))
    return out


# ---- kernel tracing (benchmarks) -------------------------------------------------------

class KernelTrace:
    """HIP event pairs around every launch of one libmdx kernel on this thread
    (mdx_trace_kernel).  Events are created here through the HIP runtime and
    recorded by libmdx on the stream each kernel is launched on."""

    _hip = None

    @classmethod
    def _hip_lib(cls):
        if cls._hip is None:
            hip = ctypes.CDLL("libamdhip64.so")
            hip.hipEventCreate.argtypes = [ctypes.POINTER(_vp)]
            hip.hipEventCreate.restype = ctypes.c_int
            hip.hipEventDestroy.argtypes = [_vp]
            hip.hipEventDestroy.restype = ctypes.c_int
            hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), _vp, _vp]
            hip.hipEventElapsedTime.restype = ctypes.c_int
            cls._hip = hip
        return cls._hip

    def __init__(self, kernel: str, capacity: int):
        hip = self._hip_lib()
        self.kernel = kernel
        self.capacity = int(capacity)
        self.starts = (_vp * self.capacity)()
        self.stops = (_vp * self.capacity)()
        for arr in (self.starts, self.stops):
            for i in range(self.capacity):
                ev = _vp()
                if hip.hipEventCreate(ctypes.byref(ev)) != 0:
                    raise RuntimeError("hipEventCreate failed")
                arr[i] = ev
        self.count = _i32(0)

    def start(self):
        self.count.value = 0
        _check(_trace(self.kernel.encode(), ctypes.cast(self.starts, _vp),
                      ctypes.cast(self.stops, _vp), self.capacity, ctypes.byref(self.count)))

    @staticmethod
    def stop_all():
        _check(_trace(None, None, None, 0, ctypes.byref(_i32(0))))

    def durations_ms(self):
        """Per-launch durations (call after the stream has synchronized)."""
        hip = self._hip_lib()
        out = []
        for i in range(min(self.count.value, self.capacity)):
            ms = ctypes.c_float(0)
            if hip.hipEventElapsedTime(ctypes.byref(ms), self.starts[i], self.stops[i]) != 0:
                raise RuntimeError("hipEventElapsedTime failed")
            out.append(float(ms.value))
        return out

    def launches(self) -> int:
        return int(self.count.value)

    def close(self):
        hip = self._hip_lib()
        for arr in (self.starts, self.stops):
            for i in range(self.capacity):
                if arr[i]:
                    hip.hipEventDestroy(arr[i])
                    arr[i] = None
