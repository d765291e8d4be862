"""MI355X (gfx950) parallel in-place merge -- Python binding.

The method is Bramas & Bramas, "On the improvement of the in-place merge
algorithm parallelization" (arXiv 2005.12648): split A|B into independent pairs
by co-rank searches (Sec. 3.1), make the pairs contiguous with in-place
partition exchanges level by level (Alg. 3, Sec. 3.4), merge every pair
independently (the per-pair merge of Alg. 2/3).

This module only marshals arguments: every step runs in the HIP kernels of
``libinplace_merge.so`` (built from ``csrc/`` by ``_build.py``) through the C
ABI declared in ``include/inplace_merge.h``.  PyTorch provides device memory and
the current stream.  There is no CPU fallback: if the library is missing or a
tensor is not on a HIP device, the call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

__all__ = [
    "IMError", "library_path", "load", "inplace_merge", "inplace_merge_kv",
    "batched_inplace_merge", "batched_inplace_merge_kv", "inplace_merge_sort",
    "corank", "rotate", "fetch_stats", "workspace_bytes", "set_workspace",
    "MergeModel", "MLP_HIDDEN", "MLP_PARAMS", "profile", "profile_read", "STAGES",
    "MergeGraph", "set_config", "autotune", "LEAF_CONFIGS",
    "inplace_merge_variant", "divide", "rotate_cs", "merge_out_of_place",
    "inplace_merge_buffered", "SPLIT_CORANK", "SPLIT_FINDMEDIAN", "ROTATE_SWAP_REV", "ROTATE_CS",
    "inplace_merge_rows", "rows_workspace_bytes", "last_stats", "device_status", "rotate_ls",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libinplace_merge.so")
_lib = None

MLP_HIDDEN = 32
MLP_PARAMS = 3 * MLP_HIDDEN + 1
LEAF_CONFIGS = 4
SPLIT_CORANK, SPLIT_FINDMEDIAN = 0, 1
ROTATE_SWAP_REV, ROTATE_CS = 0, 1
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED_DTYPE, ERR_HIP = 0, -1, -2, -3
ERR_WORKSPACE, ERR_NOT_SORTED, ERR_UNIMPLEMENTED, ERR_DEVICE = -4, -5, -6, -7

# im_dtype codes of the C ABI
_DT = {torch.int32: 0, torch.uint32: 1, torch.int64: 2, torch.uint64: 3}

_STATUS = {
    0: "IM_OK", -1: "IM_ERR_INVALID_ARG", -2: "IM_ERR_UNSUPPORTED_DTYPE", -3: "IM_ERR_HIP",
    -4: "IM_ERR_WORKSPACE", -5: "IM_ERR_NOT_SORTED", -6: "IM_ERR_UNIMPLEMENTED",
    -7: "IM_ERR_DEVICE",
}


class IMError(RuntimeError):
    """A C ABI call returned a negative status."""

    def __init__(self, code: int, msg: str):
        self.code = code
        super().__init__("%s (%d): %s" % (_STATUS.get(code, "?"), code, msg))


class _Stats(ctypes.Structure):
    _fields_ = [
        ("leaf_capacity", ctypes.c_int64), ("tile", ctypes.c_int64),
        ("max_levels", ctypes.c_int32), ("levels_used", ctypes.c_int32),
        ("leaves", ctypes.c_int64), ("tiles", ctypes.c_int64),
        ("rotations", ctypes.c_int64), ("rotated_elems", ctypes.c_int64),
        ("reversed_elems", ctypes.c_int64), ("leaf_elems", ctypes.c_int64),
        ("search_probes", ctypes.c_int64), ("searches", ctypes.c_int64),
        ("leaf_config", ctypes.c_int32), ("leaf_grid", ctypes.c_int32),
        ("split_fallbacks", ctypes.c_int64), ("fused_nodes", ctypes.c_int64),
    ]


class _TrainCfg(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int64), ("steps", ctypes.c_int32),
                ("lr", ctypes.c_float), ("seed", ctypes.c_uint64)]


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            "libinplace_merge.so is not built (%s); run __graft_entry__.build() or "
            "python -m paper_2005_12648_amd._build" % _LIB_PATH)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    sig = {
        "inplace_merge": [vp, i64, i64, c_int, vp],
        "inplace_merge_noalloc": [vp, i64, i64, c_int, vp],
        "inplace_merge_kv": [vp, vp, i64, i64, c_int, c_int, vp],
        "inplace_merge_rows": [vp, i64, i64, i64, c_int, vp],
        "batched_inplace_merge": [vp, vp, i64, c_int, vp],
        "batched_inplace_merge_kv": [vp, vp, vp, i64, c_int, c_int, vp],
        "batched_inplace_merge_sized": [vp, vp, i64, i64, i64, c_int, vp],
        "batched_inplace_merge_kv_sized": [vp, vp, vp, i64, i64, i64, c_int, c_int, vp],
        "inplace_merge_sort": [vp, i64, c_int, vp],
        "inplace_merge_set_workspace": [vp, ctypes.c_size_t],
        "inplace_merge_fetch_stats": [ctypes.POINTER(_Stats), vp],
        "inplace_merge_last_stats": [ctypes.POINTER(_Stats)],
        "inplace_merge_device_status": [],
        "im_corank": [vp, i64, i64, c_int, vp, i64, vp, vp, vp],
        "im_rotate": [vp, i64, i64, c_int, vp],
        "merge_model_create": [ctypes.POINTER(vp), vp, ctypes.c_uint64],
        "merge_model_train": [ctypes.POINTER(vp), vp, i64, i64, c_int, ctypes.POINTER(_TrainCfg), vp],
        "merge_model_grad": [vp, vp, vp, i64, vp, vp, vp],
        "merge_model_forward": [vp, vp, i64, vp, vp],
        "merge_model_get_params": [vp, vp],
        "merge_model_adam_step": [vp, vp, vp, vp, ctypes.c_float, c_int, vp],
        "merge_model_set_params": [vp, vp],
        "im_corank_learned": [vp, i64, i64, c_int, vp, vp, i64, vp, vp, vp],
        "inplace_merge_learned": [vp, i64, i64, c_int, vp, vp],
        "merge_model_save": [vp, ctypes.c_char_p],
        "merge_model_load": [ctypes.POINTER(vp), ctypes.c_char_p],
        "merge_model_free": [vp],
        "inplace_merge_profile": [c_int],
        "inplace_merge_profile_read": [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), c_int, vp],
        "batched_inplace_merge_graph": [ctypes.POINTER(vp), vp, vp, i64, i64, i64, c_int, vp],
        "im_graph_launch": [vp, vp],
        "im_graph_cooperative": [vp],
        "im_graph_destroy": [vp],
        "inplace_merge_set_config": [c_int],
        "inplace_merge_variant": [vp, i64, i64, c_int, c_int, c_int, vp],
        "im_divide": [vp, i64, i64, c_int, c_int, c_int, vp, vp],
        "im_rotate_cs": [vp, i64, i64, c_int, vp],
        "im_rotate_ls": [vp, i64, i64, c_int, vp, vp],
        "merge_out_of_place": [vp, vp, i64, i64, c_int, vp],
        "inplace_merge_buffered": [vp, i64, i64, c_int, vp],
        "inplace_merge_autotune": [vp, vp, i64, i64, i64, c_int, c_int, c_int,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_int), vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = c_int
    lib.inplace_merge_workspace_bytes.argtypes = [i64, c_int]
    lib.inplace_merge_workspace_bytes.restype = ctypes.c_size_t
    lib.inplace_merge_workspace_bytes_batched.argtypes = [i64, i64, c_int]
    lib.inplace_merge_workspace_bytes_batched.restype = ctypes.c_size_t
    lib.inplace_merge_rows_workspace_bytes.argtypes = [i64, i64, c_int]
    lib.inplace_merge_rows_workspace_bytes.restype = ctypes.c_size_t
    lib.inplace_merge_last_error.argtypes = []
    lib.inplace_merge_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        msg = load().inplace_merge_last_error()
        raise IMError(rc, msg.decode() if msg else "")


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_tensor(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must live on a HIP device (no CPU path exists)" % name)
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous 1-D tensor" % name)


def _key_code(t: torch.Tensor) -> int:
    try:
        return _DT[t.dtype]
    except KeyError:
        raise TypeError("unsupported dtype %s (int32, uint32, int64, uint64)" % t.dtype) from None


def inplace_merge(data: torch.Tensor, la: int, stream=None) -> torch.Tensor:
    """Merge data[:la] and data[la:] (two ascending runs) in place; returns data."""
    _dev_tensor(data, "data")
    n = data.numel()
    if not 0 <= la <= n:
        raise ValueError("la out of range")
    with torch.cuda.device(data.device):
        _check(load().inplace_merge(ctypes.c_void_p(data.data_ptr()), la, n - la,
                                    _key_code(data), _stream(stream)))
    return data


def inplace_merge_kv(keys: torch.Tensor, vals: torch.Tensor, la: int, stream=None):
    """Stable key+payload merge in place; returns (keys, vals)."""
    _dev_tensor(keys, "keys")
    _dev_tensor(vals, "vals")
    n = keys.numel()
    if vals.numel() != n or not 0 <= la <= n:
        raise ValueError("shape mismatch")
    with torch.cuda.device(keys.device):
        _check(load().inplace_merge_kv(ctypes.c_void_p(keys.data_ptr()),
                                       ctypes.c_void_p(vals.data_ptr()), la, n - la,
                                       _key_code(keys), _key_code(vals), _stream(stream)))
    return keys, vals


def inplace_merge_rows(rows: torch.Tensor, la: int, stream=None) -> torch.Tensor:
    """Stable in-place merge of the rows of a contiguous 2-D tensor (n, w):
    rows[:la] and rows[la:] are ascending by column 0 (the key, of the
    tensor's dtype); every row moves as a whole.  Returns rows."""
    if not isinstance(rows, torch.Tensor):
        raise TypeError("rows must be a torch.Tensor")
    if not rows.is_cuda:
        raise ValueError("rows must live on a HIP device (no CPU path exists)")
    if rows.dim() != 2 or not rows.is_contiguous():
        raise ValueError("rows must be a contiguous 2-D tensor")
    n = rows.shape[0]
    if not 0 <= la <= n:
        raise ValueError("la out of range")
    row_bytes = rows.shape[1] * rows.element_size()
    with torch.cuda.device(rows.device):
        _check(load().inplace_merge_rows(ctypes.c_void_p(rows.data_ptr()), la, n - la,
                                         row_bytes, _key_code(rows), _stream(stream)))
    return rows


def rows_workspace_bytes(rows: int, row_bytes: int, key_dtype=torch.int32) -> int:
    """Workspace bytes of a rows merge (0 if the arguments are invalid)."""
    return int(load().inplace_merge_rows_workspace_bytes(rows, row_bytes, _DT[key_dtype]))


def batched_inplace_merge(data: torch.Tensor, offsets: torch.Tensor, max_instance: int = 0,
                          stream=None, sized: bool = True) -> torch.Tensor:
    """offsets: device int64[2n+1]; instance q merges [o[2q],o[2q+1]) with [o[2q+1],o[2q+2]).

    sized=True calls batched_inplace_merge_sized with total = data.numel()
    (asynchronous); sized=False calls batched_inplace_merge, which reads the
    total back from the offsets (one synchronisation)."""
    _dev_tensor(data, "data")
    _dev_tensor(offsets, "offsets")
    if offsets.dtype != torch.int64 or offsets.numel() < 1 or offsets.numel() % 2 != 1:
        raise ValueError("offsets must be int64 with 2n+1 entries")
    n = (offsets.numel() - 1) // 2
    with torch.cuda.device(data.device):
        if sized:
            _check(load().batched_inplace_merge_sized(
                ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n,
                data.numel(), max_instance, _key_code(data), _stream(stream)))
        else:
            _check(load().batched_inplace_merge(
                ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n,
                _key_code(data), _stream(stream)))
    return data


def batched_inplace_merge_kv(keys: torch.Tensor, vals: torch.Tensor, offsets: torch.Tensor,
                             max_instance: int = 0, stream=None, sized: bool = True):
    _dev_tensor(keys, "keys")
    _dev_tensor(vals, "vals")
    _dev_tensor(offsets, "offsets")
    if offsets.dtype != torch.int64 or offsets.numel() % 2 != 1:
        raise ValueError("offsets must be int64 with 2n+1 entries")
    if vals.numel() != keys.numel():
        raise ValueError("shape mismatch")
    n = (offsets.numel() - 1) // 2
    with torch.cuda.device(keys.device):
        if sized:
            _check(load().batched_inplace_merge_kv_sized(
                ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
                ctypes.c_void_p(offsets.data_ptr()), n, keys.numel(), max_instance,
                _key_code(keys), _key_code(vals), _stream(stream)))
        else:
            _check(load().batched_inplace_merge_kv(
                ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
                ctypes.c_void_p(offsets.data_ptr()), n, _key_code(keys), _key_code(vals),
                _stream(stream)))
    return keys, vals


def inplace_merge_sort(data: torch.Tensor, stream=None) -> torch.Tensor:
    """Sort data in place: LDS tile sort, then bottom-up batched in-place merges."""
    _dev_tensor(data, "data")
    with torch.cuda.device(data.device):
        _check(load().inplace_merge_sort(ctypes.c_void_p(data.data_ptr()), data.numel(),
                                         _key_code(data), _stream(stream)))
    return data


def corank(data: torch.Tensor, la: int, ks: torch.Tensor, stream=None, probes: bool = False):
    """Co-rank i(k) of each diagonal in ks (device int64) for runs data[:la], data[la:].

    With probes=True also returns the key pairs compared per diagonal (int32)."""
    _dev_tensor(data, "data")
    _dev_tensor(ks, "ks")
    if ks.dtype != torch.int64:
        raise TypeError("ks must be int64")
    out = torch.empty_like(ks)
    pr = torch.empty(ks.numel(), dtype=torch.int32, device=ks.device) if probes else None
    n = data.numel()
    with torch.cuda.device(data.device):
        _check(load().im_corank(ctypes.c_void_p(data.data_ptr()), la, n - la, _key_code(data),
                                ctypes.c_void_p(ks.data_ptr()), ks.numel(),
                                ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(pr.data_ptr()) if probes else None,
                                _stream(stream)))
    return (out, pr) if probes else out


def rotate(data: torch.Tensor, lx: int, stream=None) -> torch.Tensor:
    """Partition exchange in place: data = X|Y with |X| = lx becomes Y|X."""
    _dev_tensor(data, "data")
    n = data.numel()
    if not 0 <= lx <= n:
        raise ValueError("lx out of range")
    with torch.cuda.device(data.device):
        _check(load().im_rotate(ctypes.c_void_p(data.data_ptr()), lx, n - lx,
                                data.element_size(), _stream(stream)))
    return data


def inplace_merge_variant(data: torch.Tensor, la: int, split: int = SPLIT_CORANK,
                          rotation: int = ROTATE_SWAP_REV, stream=None) -> torch.Tensor:
    """In-place merge with the split (co-rank / FindMedian) and exchange (linear /
    circular shifting) methods of the paper chosen; keys only."""
    _dev_tensor(data, "data")
    n = data.numel()
    if not 0 <= la <= n:
        raise ValueError("la out of range")
    with torch.cuda.device(data.device):
        _check(load().inplace_merge_variant(ctypes.c_void_p(data.data_ptr()), la, n - la,
                                            _key_code(data), int(split), int(rotation),
                                            _stream(stream)))
    return data


def divide(data: torch.Tensor, la: int, depth: int, method: int = SPLIT_CORANK,
           stream=None) -> torch.Tensor:
    """Pair sizes (|A_p|, |B_p|) of the recursive division into 2**depth pairs
    (no data movement); int64 device tensor of shape (2**depth, 2)."""
    _dev_tensor(data, "data")
    n = data.numel()
    if not 0 <= la <= n:
        raise ValueError("la out of range")
    out = torch.empty((1 << depth, 2), dtype=torch.int64, device=data.device)
    with torch.cuda.device(data.device):
        _check(load().im_divide(ctypes.c_void_p(data.data_ptr()), la, n - la, _key_code(data),
                                int(method), int(depth), ctypes.c_void_p(out.data_ptr()),
                                _stream(stream)))
    return out


def rotate_cs(data: torch.Tensor, lx: int, stream=None) -> torch.Tensor:
    """Partition exchange by circular shifting: data = X|Y becomes Y|X."""
    _dev_tensor(data, "data")
    n = data.numel()
    if not 0 <= lx <= n:
        raise ValueError("lx out of range")
    with torch.cuda.device(data.device):
        _check(load().im_rotate_cs(ctypes.c_void_p(data.data_ptr()), lx, n - lx,
                                   data.element_size(), _stream(stream)))
    return data


def rotate_ls(data: torch.Tensor, lx: int, stream=None, count: bool = True):
    """Partition exchange by linear shifting, step by step (the paper's swaps):
    data = X|Y becomes Y|X.  Returns (data, element swaps counted on the
    device, read after a synchronisation of the stream), or (data, None)
    with count=False (no count, no synchronisation)."""
    _dev_tensor(data, "data")
    n = data.numel()
    if not 0 <= lx <= n:
        raise ValueError("lx out of range")
    swaps = torch.zeros(1, dtype=torch.int64, device=data.device) if count else None
    with torch.cuda.device(data.device):
        _check(load().im_rotate_ls(ctypes.c_void_p(data.data_ptr()), lx, n - lx,
                                   data.element_size(),
                                   ctypes.c_void_p(swaps.data_ptr()) if count else None,
                                   _stream(stream)))
    return data, (int(swaps.item()) if count else None)


def merge_out_of_place(data: torch.Tensor, la: int, out: Optional[torch.Tensor] = None,
                       stream=None) -> torch.Tensor:
    """Stable merge of data[:la] and data[la:] into a separate tensor."""
    _dev_tensor(data, "data")
    n = data.numel()
    if not 0 <= la <= n:
        raise ValueError("la out of range")
    if out is None:
        out = torch.empty_like(data)
    _dev_tensor(out, "out")
    if out.numel() != n or out.dtype != data.dtype:
        raise ValueError("out must match data")
    with torch.cuda.device(data.device):
        _check(load().merge_out_of_place(ctypes.c_void_p(data.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), la, n - la,
                                         _key_code(data), _stream(stream)))
    return out


def inplace_merge_buffered(data: torch.Tensor, la: int, stream=None) -> torch.Tensor:
    """Merge through a temporary buffer (allocate, merge, copy back, free)."""
    _dev_tensor(data, "data")
    n = data.numel()
    if not 0 <= la <= n:
        raise ValueError("la out of range")
    with torch.cuda.device(data.device):
        _check(load().inplace_merge_buffered(ctypes.c_void_p(data.data_ptr()), la, n - la,
                                             _key_code(data), _stream(stream)))
    return data


def fetch_stats(stream=None) -> dict:
    """Statistics of the last merge enqueued by this thread (synchronises the stream)."""
    st = _Stats()
    _check(load().inplace_merge_fetch_stats(ctypes.byref(st), _stream(stream)))
    return {f: getattr(st, f) for f, _ in _Stats._fields_}


def last_stats() -> dict:
    """Statistics of the last merge of this thread (synchronises the stream it ran on)."""
    st = _Stats()
    _check(load().inplace_merge_last_stats(ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in _Stats._fields_}


def device_status(device=None) -> int:
    """Device-side error bits raised since the last query on this device, read
    without a synchronisation: raises IMError(ERR_DEVICE) if any, else 0."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    with torch.cuda.device(dev):
        _check(load().inplace_merge_device_status())
    return 0


STAGES = ("split", "rotate", "plan", "tilerank", "leafmerge")


def profile(enable: bool):
    """Record per-stage HIP events on the merge's stream (this thread)."""
    _check(load().inplace_merge_profile(1 if enable else 0))


def profile_read(stream=None) -> dict:
    """{stage: (ms, launches)} accumulated since the last read (synchronises)."""
    ms = (ctypes.c_double * len(STAGES))()
    ln = (ctypes.c_int64 * len(STAGES))()
    _check(load().inplace_merge_profile_read(ms, ln, len(STAGES), _stream(stream)))
    return {s: (ms[i], ln[i]) for i, s in enumerate(STAGES)}


def workspace_bytes(total_elems: int, n_inst: int, dtype: torch.dtype) -> int:
    """Workspace bytes of a merge of total_elems elements in n_inst instances
    (n_inst == 1: any single merge or merge sort of that length)."""
    if n_inst == 1:
        return int(load().inplace_merge_workspace_bytes(total_elems, _DT[dtype]))
    return int(load().inplace_merge_workspace_bytes_batched(total_elems, n_inst, _DT[dtype]))


def set_workspace(buf: Optional[torch.Tensor]):
    """Use a caller-owned device buffer as the workspace of its device (None: library-owned)."""
    if buf is None:
        _check(load().inplace_merge_set_workspace(None, 0))
        return
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    with torch.cuda.device(buf.device):
        _check(load().inplace_merge_set_workspace(ctypes.c_void_p(buf.data_ptr()),
                                                  buf.numel() * buf.element_size()))


class MergeGraph:
    """A batched merge recorded once in a HIP graph and replayed by launch().

    The data and offsets tensors are baked into the graph: keep them alive and
    change only their contents between replays (same instance count, total at
    most ``data.numel()``, every instance at most ``max_instance``)."""

    def __init__(self, data: torch.Tensor, offsets: torch.Tensor, max_instance: int = 0,
                 stream=None):
        _dev_tensor(data, "data")
        _dev_tensor(offsets, "offsets")
        if offsets.dtype != torch.int64 or offsets.numel() < 3 or offsets.numel() % 2 != 1:
            raise ValueError("offsets must be int64 with 2n+1 entries, n >= 1")
        self._h = None
        self._data, self._offsets = data, offsets
        h = ctypes.c_void_p()
        n = (offsets.numel() - 1) // 2
        with torch.cuda.device(data.device):
            _check(load().batched_inplace_merge_graph(
                ctypes.byref(h), ctypes.c_void_p(data.data_ptr()),
                ctypes.c_void_p(offsets.data_ptr()), n, data.numel(), max_instance,
                _key_code(data), _stream(stream)))
        self._h = h
        self.device = data.device

    @property
    def cooperative(self) -> bool:
        return bool(load().im_graph_cooperative(self._h))

    def launch(self, stream=None):
        with torch.cuda.device(self.device):
            _check(load().im_graph_launch(self._h, _stream(stream)))
        return self._data

    def close(self):
        if self._h is not None and _lib is not None:
            with torch.cuda.device(self.device):
                load().im_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_config(cfg: int):
    """Force the leaf-merge configuration (0..LEAF_CONFIGS-1) or -1 for automatic."""
    _check(load().inplace_merge_set_config(int(cfg)))


def autotune(data: torch.Tensor, offsets: torch.Tensor, max_instance: int = 0,
             vals_dtype: Optional[torch.dtype] = None, reps: int = 3, stream=None):
    """Time every leaf configuration on a copy of this batched input and remember
    the fastest for its workload class.  Returns (chosen, [median ms per config])."""
    _dev_tensor(data, "data")
    _dev_tensor(offsets, "offsets")
    if offsets.dtype != torch.int64 or offsets.numel() < 3 or offsets.numel() % 2 != 1:
        raise ValueError("offsets must be int64 with 2n+1 entries, n >= 1")
    n = (offsets.numel() - 1) // 2
    ms = (ctypes.c_double * LEAF_CONFIGS)()
    chosen = ctypes.c_int(-1)
    vcode = -1 if vals_dtype is None else _DT[vals_dtype]
    with torch.cuda.device(data.device):
        _check(load().inplace_merge_autotune(
            ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n,
            data.numel(), max_instance, _key_code(data), vcode, reps, ms, ctypes.byref(chosen),
            _stream(stream)))
    return chosen.value, list(ms)


class MergeModel:
    """Learned split: a 1->32->1 ReLU network (fp32) that predicts co-ranks.

    Not part of the paper.  Predictions are always corrected to the exact
    co-rank by an exponential-then-binary search, so merges are bit-identical
    to the plain method."""

    def __init__(self, params=None, seed: int = 0, _handle=None):
        lib = load()
        if _handle is not None:
            self._h = _handle
            return
        h = ctypes.c_void_p()
        if params is not None:
            p = torch.as_tensor(params, dtype=torch.float32).contiguous().cpu()
            if p.numel() != MLP_PARAMS:
                raise ValueError("expected %d parameters" % MLP_PARAMS)
            _check(lib.merge_model_create(ctypes.byref(h), ctypes.c_void_p(p.data_ptr()), seed))
        else:
            _check(lib.merge_model_create(ctypes.byref(h), None, seed))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.merge_model_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def params(self) -> torch.Tensor:
        p = torch.empty(MLP_PARAMS, dtype=torch.float32)
        _check(load().merge_model_get_params(self._h, ctypes.c_void_p(p.data_ptr())))
        return p

    def set_params(self, params):
        p = torch.as_tensor(params, dtype=torch.float32).contiguous().cpu()
        _check(load().merge_model_set_params(self._h, ctypes.c_void_p(p.data_ptr())))

    def train(self, data: torch.Tensor, la: int, samples: int = 4096, steps: int = 2000,
              lr: float = 3e-3, seed: int = 0, stream=None):
        _dev_tensor(data, "data")
        cfg = _TrainCfg(samples, steps, lr, seed)
        with torch.cuda.device(data.device):
            _check(load().merge_model_train(ctypes.byref(self._h), ctypes.c_void_p(data.data_ptr()),
                                            la, data.numel() - la, _key_code(data),
                                            ctypes.byref(cfg), _stream(stream)))
        return self

    def grad(self, x: torch.Tensor, t: torch.Tensor, stream=None):
        """(gradient[97], loss) of the mean squared error on device samples x, t (fp32)."""
        _dev_tensor(x, "x")
        _dev_tensor(t, "t")
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        with torch.cuda.device(x.device):
            _check(load().merge_model_grad(self._h, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(t.data_ptr()), x.numel(),
                                           ctypes.c_void_p(g.data_ptr()),
                                           ctypes.c_void_p(loss.data_ptr()), _stream(stream)))
        return g, loss

    def adam_step(self, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr: float, step: int,
                  stream=None):
        """One Adam step of the device parameters with device gradient g; the
        moments m, v (device fp32, MLP_PARAMS each) are updated in place."""
        for t, name in ((g, "g"), (m, "m"), (v, "v")):
            _dev_tensor(t, name)
            if t.dtype != torch.float32 or t.numel() != MLP_PARAMS:
                raise ValueError("%s must be float32 with %d entries" % (name, MLP_PARAMS))
        with torch.cuda.device(g.device):
            _check(load().merge_model_adam_step(self._h, ctypes.c_void_p(g.data_ptr()),
                                                ctypes.c_void_p(m.data_ptr()),
                                                ctypes.c_void_p(v.data_ptr()), float(lr),
                                                int(step), _stream(stream)))

    def forward(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        _dev_tensor(x, "x")
        y = torch.empty_like(x)
        with torch.cuda.device(x.device):
            _check(load().merge_model_forward(self._h, ctypes.c_void_p(x.data_ptr()), x.numel(),
                                              ctypes.c_void_p(y.data_ptr()), _stream(stream)))
        return y

    def corank(self, data: torch.Tensor, la: int, ks: torch.Tensor, stream=None):
        """Learned co-ranks (exact) and probes per diagonal."""
        _dev_tensor(data, "data")
        _dev_tensor(ks, "ks")
        out = torch.empty_like(ks)
        probes = torch.empty(ks.numel(), dtype=torch.int32, device=ks.device)
        with torch.cuda.device(data.device):
            _check(load().im_corank_learned(ctypes.c_void_p(data.data_ptr()), la,
                                            data.numel() - la, _key_code(data), self._h,
                                            ctypes.c_void_p(ks.data_ptr()), ks.numel(),
                                            ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(probes.data_ptr()), _stream(stream)))
        return out, probes

    def merge(self, data: torch.Tensor, la: int, stream=None) -> torch.Tensor:
        _dev_tensor(data, "data")
        with torch.cuda.device(data.device):
            _check(load().inplace_merge_learned(ctypes.c_void_p(data.data_ptr()), la,
                                                data.numel() - la, _key_code(data), self._h,
                                                _stream(stream)))
        return data

    def save(self, path: str):
        _check(load().merge_model_save(self._h, path.encode()))

    @classmethod
    def load_file(cls, path: str) -> "MergeModel":
        h = ctypes.c_void_p()
        _check(load().merge_model_load(ctypes.byref(h), path.encode()))
        return cls(_handle=h)
