"""Thin ctypes binding of the C ABI in include/ph0.h (same names).

Only argument marshalling lives here: every step of the barcode computation
runs in the HIP kernels of libph0.so.  There is no CPU fallback: loading
fails loudly when the library has not been built.

Device entry points take torch tensors on a HIP device and enqueue on the
current torch stream (or the one given); host entry points take numpy.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libph0.so")

PH0_INF = 0xFFFFFFFF
PH0_I8 = 1
PH0_I16 = 2
STATUS = {0: "PH0_OK", -1: "PH0_EINVAL", -2: "PH0_ERANGE", -3: "PH0_ENOMEM",
          -4: "PH0_EDEVICE", -5: "PH0_EBUSY"}


class Ph0Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class ph0_stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("E", ctypes.c_int64),
        ("E_eff", ctypes.c_int64),
        ("distinct_eff", ctypes.c_int64),
        ("additions", ctypes.c_int64),
        ("additions_all", ctypes.c_int64),
        ("find_steps", ctypes.c_int64),
        ("words_read", ctypes.c_int64),
        ("rounds", ctypes.c_int64),
        ("window", ctypes.c_int64),
        ("sort_passes", ctypes.c_int32),
        ("delta_bits", ctypes.c_int32),
        ("index_bits", ctypes.c_int32),
        ("keys_path", ctypes.c_int32),
        ("ms_keys", ctypes.c_float),
        ("ms_sort", ctypes.c_float),
        ("ms_reduce", ctypes.c_float),
        ("ms_rank", ctypes.c_float),
        ("ms_emit", ctypes.c_float),
        ("ms_total", ctypes.c_float),
        ("ms_walk_kernel", ctypes.c_float),
        ("ms_radix_kernel", ctypes.c_float),
        ("walk_launches", ctypes.c_int32),
        ("radix_launches", ctypes.c_int32),
        ("sort_chunks", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("sorted_keys", ctypes.c_int64),
    ]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ph0_h1_stats(ctypes.Structure):
    _fields_ = [
        ("E", ctypes.c_int64),
        ("T", ctypes.c_int64),
        ("pivots", ctypes.c_int64),
        ("emergent", ctypes.c_int64),
        ("bars", ctypes.c_int64),
        ("zero_length", ctypes.c_int64),
        ("additions", ctypes.c_int64),
        ("rounds", ctypes.c_int64),
        ("walks", ctypes.c_int64),
        ("ms_setup", ctypes.c_float),
        ("ms_reduce", ctypes.c_float),
        ("ms_total", ctypes.c_float),
        ("reserved", ctypes.c_int32),
    ]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SIGS = {
    "ph0_last_error": ([], ctypes.c_char_p),
    "ph0_workspace_bytes": ([_I64, _I32, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "ph0_key_layout": ([_I64, _I32, ctypes.c_int, ctypes.POINTER(_I32), ctypes.POINTER(_I32)], ctypes.c_int),
    "ph0_set_window": ([_I64], ctypes.c_int),
    "ph0_workspace_bytes_f32": ([_I64, _I32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "ph0_barcodes_f32_device": ([_P, _I64, _I32, ctypes.c_double, ctypes.c_double, _P, _P,
                                 ctypes.c_size_t, _P, ctypes.POINTER(ph0_stats)], ctypes.c_int),
    "ph0_barcodes": ([_P, ctypes.c_int, _I64, _I32, _P, ctypes.POINTER(ph0_stats)], ctypes.c_int),
    "ph0_barcodes_device": ([_P, ctypes.c_int, _I64, _I32, _P, _P, ctypes.c_size_t, _P,
                             ctypes.POINTER(ph0_stats)], ctypes.c_int),
    "ph0_pairs_device": ([_P, ctypes.c_int, _I64, _I32, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P,
                          ctypes.POINTER(ph0_stats)], ctypes.c_int),
    "ph0_batched_workspace_bytes": ([_P, _I64, _I32, ctypes.c_int, _P, ctypes.POINTER(ctypes.c_size_t)],
                                    ctypes.c_int),
    "ph0_barcodes_batched_device": ([_P, ctypes.c_int, _P, _I64, _I32, _P, _P, ctypes.c_size_t, _P, _P,
                                     ctypes.POINTER(ph0_stats)], ctypes.c_int),
    "ph0_barcodes_batched": ([_P, ctypes.c_int, _P, _I64, _I32, _P, ctypes.c_char_p,
                              ctypes.POINTER(ph0_stats)], ctypes.c_int),
    "ph0_barcodes_batched_device_noalloc": ([_P, ctypes.c_int, _P, _I64, _I32, _P, _P, _P],
                                            ctypes.c_int),
    "ph0_server_create": ([ctypes.c_size_t, _I32, ctypes.POINTER(_P)], ctypes.c_int),
    "ph0_server_request_bytes": ([_I64, _I32, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "ph0_server_submit": ([_P, _P, ctypes.c_int, _I64, _I32, ctypes.c_uint64], ctypes.c_int),
    "ph0_server_poll": ([_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_I32), _P, _I64,
                         ctypes.POINTER(_I64)], ctypes.c_int),
    "ph0_server_in_flight": ([_P], _I64),
    "ph0_server_destroy": ([_P], None),
    "ph0_keys_device": ([_P, ctypes.c_int, _I64, _I32, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "ph0_sorted_keys_device": ([_P, ctypes.c_int, _I64, _I32, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "ph0_h1_workspace_bytes": ([_I64, _I32, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "ph0_h1_device": ([_P, ctypes.c_int, _I64, _I32, _P, _P, ctypes.POINTER(_I64), _P, ctypes.c_size_t,
                       _P, ctypes.POINTER(ph0_h1_stats)], ctypes.c_int),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libph0.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libph0.so is not built; run `python -m paper_2203_02527_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def ph0_last_error() -> str:
    return lib().ph0_last_error().decode()


def _check(rc: int):
    if rc != 0:
        raise Ph0Error(rc, ph0_last_error())


def _dtype_code(dtype) -> int:
    s = str(dtype).replace("<class '", "").rstrip("'>")
    if s.endswith("uint8") or s.endswith("uint16"):
        raise TypeError("points must be signed int8 or int16, got %s" % s)
    if s.endswith("int8"):
        return PH0_I8
    if s.endswith("int16"):
        return PH0_I16
    raise TypeError("points must be int8 or int16, got %s" % s)


def ph0_workspace_bytes(n: int, d: int, dtype) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().ph0_workspace_bytes(n, d, _dtype_code(dtype), ctypes.byref(out)))
    return out.value


def ph0_key_layout(n: int, d: int, dtype) -> tuple[int, int, int]:
    """(status, index_bits, delta_bits) for full-range coordinates."""
    ib, db = _I32(0), _I32(0)
    rc = lib().ph0_key_layout(n, d, _dtype_code(dtype), ctypes.byref(ib), ctypes.byref(db))
    return rc, ib.value, db.value


def ph0_set_window(columns: int) -> None:
    _check(lib().ph0_set_window(columns))


def ph0_barcodes(points: np.ndarray, with_stats: bool = False):
    """Host API: N x d int8/int16 numpy array -> N x 2 uint32 (birth, death)."""
    x = np.ascontiguousarray(points)
    if x.ndim != 2:
        raise ValueError("points must be N x d")
    n, d = x.shape
    out = np.empty((n, 2), np.uint32)
    # No statistics asked: NULL, so that small clouds take the one-workgroup route.
    st = ph0_stats()
    _check(lib().ph0_barcodes(x.ctypes.data_as(_P), _dtype_code(x.dtype), n, d,
                              out.ctypes.data_as(_P), ctypes.byref(st) if with_stats else None))
    return (out, st.to_dict()) if with_stats else out


# ---- device (torch) entry points ----

def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _points_dev(points):
    if not points.is_cuda:
        raise ValueError("points must be a device tensor")
    if points.dim() != 2:
        raise ValueError("points must be N x d")
    return points.contiguous()


def alloc_workspace(n: int, d: int, dtype, device=None):
    """A byte tensor large enough for ph0_barcodes_device on this cloud shape."""
    torch = _torch()
    nbytes = ph0_workspace_bytes(n, d, dtype)
    return torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def ph0_barcodes_device(points, out=None, workspace=None, stream=None, with_stats=False):
    """Device API: returns an N x 2 int32 tensor holding the uint32 bars.

    View it as uint32 on the host (``out.cpu().numpy().view(np.uint32)``);
    PH0_INF reads as -1 in int32.
    """
    torch = _torch()
    x = _points_dev(points)
    n, d = x.shape
    if out is None:
        out = torch.empty((n, 2), dtype=torch.int32, device=x.device)
    if workspace is None:
        workspace = alloc_workspace(n, d, x.dtype, x.device)
    # No statistics asked: NULL, so that small clouds take the one-workgroup route.
    st = ph0_stats()
    _check(lib().ph0_barcodes_device(_ptr(x), _dtype_code(x.dtype), n, d, _ptr(out),
                                     _ptr(workspace), workspace.numel(), _stream_ptr(stream),
                                     ctypes.byref(st) if with_stats else None))
    return (out, st.to_dict()) if with_stats else out


def ph0_workspace_bytes_f32(n: int, d: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().ph0_workspace_bytes_f32(n, d, ctypes.byref(b)))
    return b.value


def ph0_barcodes_f32_device(points, lo: float, hi: float, out=None, workspace=None, stream=None,
                            with_stats=False):
    """Real-valued points (float32 device tensor, N x d, every coordinate in
    [lo, hi]): the barcode of their int16 grid cloud (see include/ph0.h).
    Returns the N x 2 int32 bars as ph0_barcodes_device does."""
    torch = _torch()
    x = _points_dev(points)
    if x.dtype != torch.float32:
        raise TypeError("points must be float32, got %s" % x.dtype)
    n, d = x.shape
    if out is None:
        out = torch.empty((n, 2), dtype=torch.int32, device=x.device)
    if workspace is None:
        workspace = torch.empty(ph0_workspace_bytes_f32(n, d), dtype=torch.uint8, device=x.device)
    st = ph0_stats()
    _check(lib().ph0_barcodes_f32_device(_ptr(x), n, d, float(lo), float(hi), _ptr(out),
                                         _ptr(workspace), workspace.numel(), _stream_ptr(stream),
                                         ctypes.byref(st) if with_stats else None))
    return (out, st.to_dict()) if with_stats else out


def ph0_h1_workspace_bytes(n: int, d: int, dtype) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().ph0_h1_workspace_bytes(n, d, _dtype_code(dtype), ctypes.byref(b)))
    return b.value


def ph0_h1_device(points, workspace=None, stream=None, with_stats=False):
    """H1 barcode (see include/ph0.h).  Returns (bars, tri_of_edge): an
    m x 2 int32 tensor of (birth, death) grades sorted by (birth, death), and
    an int64 tensor of E entries (the triangle paired with each sorted edge
    position, -1 if none); with_stats adds the statistics dict."""
    torch = _torch()
    x = _points_dev(points)
    n, d = x.shape
    E = n * (n - 1) // 2
    cap = max(E - n + 1, 1)
    bars = torch.empty((cap, 2), dtype=torch.int32, device=x.device)
    toe = torch.empty(max(E, 1), dtype=torch.int64, device=x.device)
    if workspace is None:
        workspace = torch.empty(ph0_h1_workspace_bytes(n, d, x.dtype), dtype=torch.uint8,
                                device=x.device)
    m = _I64(0)
    st = ph0_h1_stats()
    _check(lib().ph0_h1_device(_ptr(x), _dtype_code(x.dtype), n, d, _ptr(bars), _ptr(toe),
                               ctypes.byref(m), _ptr(workspace), workspace.numel(),
                               _stream_ptr(stream), ctypes.byref(st)))
    out = (bars[: m.value], toe[:E])
    return (*out, st.to_dict()) if with_stats else out


@dataclass
class Pairs:
    death_by_vertex: object  # int32 tensor holding uint32 grades (PH0_INF = -1)
    killer_pos: object       # int64
    killer_edge: object      # int64 holding (j << 32) | i
    killer_sqdist: object    # int64
    partner: object          # int32
    stats: dict


def ph0_pairs_device(points, workspace=None, stream=None) -> Pairs:
    torch = _torch()
    x = _points_dev(points)
    n, d = x.shape
    dev = x.device
    dbv = torch.empty(n, dtype=torch.int32, device=dev)
    kp = torch.empty(n, dtype=torch.int64, device=dev)
    ke = torch.empty(n, dtype=torch.int64, device=dev)
    ks = torch.empty(n, dtype=torch.int64, device=dev)
    par = torch.empty(n, dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = alloc_workspace(n, d, x.dtype, dev)
    st = ph0_stats()
    _check(lib().ph0_pairs_device(_ptr(x), _dtype_code(x.dtype), n, d, _ptr(dbv), _ptr(kp),
                                  _ptr(ke), _ptr(ks), _ptr(par), _ptr(workspace),
                                  workspace.numel(), _stream_ptr(stream), ctypes.byref(st)))
    return Pairs(dbv, kp, ke, ks, par, st.to_dict())


def ph0_keys_device(points, workspace=None, stream=None):
    """Unsorted packed keys (int64 tensor of E entries, colex order)."""
    torch = _torch()
    x = _points_dev(points)
    n, d = x.shape
    keys = torch.empty(max(n * (n - 1) // 2, 1), dtype=torch.int64, device=x.device)
    if workspace is None:
        workspace = alloc_workspace(n, d, x.dtype, x.device)
    _check(lib().ph0_keys_device(_ptr(x), _dtype_code(x.dtype), n, d, _ptr(keys),
                                 _ptr(workspace), workspace.numel(), _stream_ptr(stream)))
    return keys[: n * (n - 1) // 2]


def ph0_sorted_keys_device(points, workspace=None, stream=None):
    """Packed keys in sorted (delta, j, i) order (int64 tensor of E entries)."""
    torch = _torch()
    x = _points_dev(points)
    n, d = x.shape
    keys = torch.empty(max(n * (n - 1) // 2, 1), dtype=torch.int64, device=x.device)
    if workspace is None:
        workspace = alloc_workspace(n, d, x.dtype, x.device)
    _check(lib().ph0_sorted_keys_device(_ptr(x), _dtype_code(x.dtype), n, d, _ptr(keys),
                                        _ptr(workspace), workspace.numel(), _stream_ptr(stream)))
    return keys[: n * (n - 1) // 2]


class ph0_batch_tuning(ctypes.Structure):
    _fields_ = [("chunk_mult", ctypes.c_int32 * 4), ("blocks_per_cu", ctypes.c_int32),
                ("digit_bits", ctypes.c_int32), ("waves_per_cloud", ctypes.c_int32)]


def make_tuning(chunk_mult=(0, 0, 0, 0), blocks_per_cu=0, digit_bits=0,
                waves_per_cloud=0) -> ph0_batch_tuning:
    t = ph0_batch_tuning()
    for k, v in enumerate(chunk_mult):
        t.chunk_mult[k] = int(v)
    t.blocks_per_cu = int(blocks_per_cu)
    t.digit_bits = int(digit_bits)
    t.waves_per_cloud = int(waves_per_cloud)
    return t


_default_tuning = None


def default_tuning():
    """The tuning table written by the autotuner (tuning/batched.json), as a
    ph0_batch_tuning, or None (the library's built-in values) if absent."""
    global _default_tuning
    if _default_tuning is None:
        from . import autotune

        t = autotune.load()
        _default_tuning = (False,) if t is None else (
            True, make_tuning(t["chunk_mult"], t["blocks_per_cu"], t.get("digit_bits", 0),
                              t.get("waves_per_cloud", 0)))
    return _default_tuning[1] if _default_tuning[0] else None


def _offsets(offsets) -> np.ndarray:
    o = np.ascontiguousarray(offsets, dtype=np.int64)
    if o.ndim != 1 or o.size < 2:
        raise ValueError("offsets must hold nclouds + 1 entries")
    return o


def ph0_batched_workspace_bytes(offsets, d: int, dtype, tuning=None) -> int:
    o = _offsets(offsets)
    tuning = default_tuning() if tuning is None else tuning
    out = ctypes.c_size_t(0)
    _check(lib().ph0_batched_workspace_bytes(o.ctypes.data_as(_P), o.size - 1, d, _dtype_code(dtype),
                                             None if tuning is None else ctypes.byref(tuning),
                                             ctypes.byref(out)))
    return out.value


def ph0_barcodes_batched_device(points, offsets, out=None, workspace=None, tuning=None,
                                stream=None, with_stats=False):
    """Barcodes of many clouds (rows offsets[c]:offsets[c+1] of `points`).

    Returns an (offsets[-1], 2) int32 tensor of uint32 bars, each cloud's
    canonical barcode in its own rows.
    """
    torch = _torch()
    x = _points_dev(points)
    o = _offsets(offsets)
    tuning = default_tuning() if tuning is None else tuning
    if int(o[-1]) != x.shape[0]:
        raise ValueError("offsets[-1] must equal the number of rows")
    d = x.shape[1]
    if out is None:
        out = torch.empty((x.shape[0], 2), dtype=torch.int32, device=x.device)
    if workspace is None:
        nbytes = ph0_batched_workspace_bytes(o, d, x.dtype, tuning)
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    st = ph0_stats()
    _check(lib().ph0_barcodes_batched_device(
        _ptr(x), _dtype_code(x.dtype), o.ctypes.data_as(_P), o.size - 1, d, _ptr(out),
        _ptr(workspace), workspace.numel(), None if tuning is None else ctypes.byref(tuning),
        _stream_ptr(stream), ctypes.byref(st)))
    return (out, st.to_dict()) if with_stats else out


def ph0_barcodes_batched_device_noalloc(points, offsets, out=None, tuning=None, stream=None):
    """ph0_barcodes_batched_device without a workspace: the library's fixed
    device array serves as one, and the C call allocates nothing (clouds
    must have n <= 512, n * d <= 8192, d <= 64).  `out` (offsets[-1] x 2
    int32 on the device) is allocated here only when not given."""
    torch = _torch()
    x = _points_dev(points)
    o = _offsets(offsets)
    tuning = default_tuning() if tuning is None else tuning
    if int(o[-1]) != x.shape[0]:
        raise ValueError("offsets[-1] must equal the number of rows")
    if out is None:
        out = torch.empty((x.shape[0], 2), dtype=torch.int32, device=x.device)
    _check(lib().ph0_barcodes_batched_device_noalloc(
        _ptr(x), _dtype_code(x.dtype), o.ctypes.data_as(_P), o.size - 1, x.shape[1], _ptr(out),
        None if tuning is None else ctypes.byref(tuning), _stream_ptr(stream)))
    return out


def _default_tune_json():
    """The autotuner's table as the tuning text ph0_barcodes_batched takes."""
    t = default_tuning()
    if t is None:
        return None
    return json.dumps({"chunk_mult": list(t.chunk_mult), "blocks_per_cu": t.blocks_per_cu,
                       "digit_bits": t.digit_bits, "waves_per_cloud": t.waves_per_cloud})


def ph0_barcodes_batched(points: np.ndarray, offsets, tune_json=None, with_stats=False):
    """Barcodes of many clouds on host memory (the library copies in and out).

    Returns an (offsets[-1], 2) uint32 array, each cloud's canonical barcode
    in its own rows.  tune_json: the tuning text (None: the autotuner's table,
    or the built-in values when there is none).
    """
    x = np.ascontiguousarray(points)
    if x.ndim != 2:
        raise ValueError("points must be a 2-D (rows, d) array")
    o = _offsets(offsets)
    if int(o[-1]) != x.shape[0]:
        raise ValueError("offsets[-1] must equal the number of rows")
    if tune_json is None:
        tune_json = _default_tune_json()
    out = np.empty((x.shape[0], 2), np.uint32)
    st = ph0_stats()
    _check(lib().ph0_barcodes_batched(
        x.ctypes.data_as(_P), _dtype_code(x.dtype), o.ctypes.data_as(_P), o.size - 1, x.shape[1],
        out.ctypes.data_as(_P), None if tune_json is None else tune_json.encode(),
        ctypes.byref(st)))
    return (out, st.to_dict()) if with_stats else out


# ---- serving ----

def ph0_server_request_bytes(n: int, d: int, dtype) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().ph0_server_request_bytes(n, d, _dtype_code(dtype), ctypes.byref(out)))
    return out.value


class Server:
    """Continuous-batching server (ph0_server_* entry points).

    submit() admits a cloud when a slot and pool memory are free (else it
    returns False: retry later); admitted clouds run concurrently on their own
    streams; poll() returns finished (tag, status, bars) without blocking.
    """

    def __init__(self, mem_budget_bytes: int, max_slots: int = 4):
        h = _P()
        _check(lib().ph0_server_create(int(mem_budget_bytes), int(max_slots), ctypes.byref(h)))
        self._h = h
        self.max_slots = max_slots
        self._buf = np.empty((65536, 2), np.uint32)

    def submit(self, points: np.ndarray, tag: int) -> bool:
        x = np.ascontiguousarray(points)
        rc = lib().ph0_server_submit(self._h, x.ctypes.data_as(_P), _dtype_code(x.dtype),
                                     x.shape[0], x.shape[1], int(tag))
        if rc == -5:
            return False
        _check(rc)
        return True

    def poll(self, max_n: int = 65536):
        tag = ctypes.c_uint64(0)
        status = _I32(0)
        n_out = _I64(0)
        buf = self._buf
        got = lib().ph0_server_poll(self._h, ctypes.byref(tag), ctypes.byref(status),
                                    buf.ctypes.data_as(_P), min(max_n, buf.shape[0]),
                                    ctypes.byref(n_out))
        if got <= 0:
            return None
        return tag.value, status.value, buf[: n_out.value].copy()

    def in_flight(self) -> int:
        return int(lib().ph0_server_in_flight(self._h))

    def close(self):
        if self._h:
            lib().ph0_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
