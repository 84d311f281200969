"""ctypes binding of libpcx.so (same names as the C ABI in include/pcx.h).

Argument marshalling only: networks are copied to the device by
``pcx_mlp_create``, the extraction runs entirely in the library's HIP kernels,
and results are copied back on request. Importing this module without the
built library raises ``ImportError``: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

# PyTorch (device memory and streams for the callers of this library) ships its
# own HIP runtime under the same soname as ROCm's. Whichever loads first serves
# the whole process, and PyTorch cannot start on another build's runtime: so
# torch, when installed, is loaded before libpcx.so, and both share its runtime.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcx.so")

PCX_OK, PCX_PENDING = 0, 1
PCX_ERR_INVALID, PCX_ERR_OOM, PCX_ERR_DEGENERATE, PCX_ERR_DEVICE, PCX_ERR_CAPACITY = -1, -2, -3, -4, -5
KERNEL_FAMILIES = ["gemm", "next", "select", "split", "sort", "pair"]
PAIRING = {"hash": 0, "sort": 1}

# every symbol include/pcx.h declares
SYMBOLS = [
    "pcx_last_error", "pcx_mlp_create", "pcx_mlp_free", "pcx_extract", "pcx_extract_simplex", "pcx_cell_counts",
    "pcx_regions", "pcx_complex_info",
    "pcx_complex_steps", "pcx_complex_copy", "pcx_complex_device", "pcx_complex_kernel_time",
    "pcx_complex_free", "pcx_cache_trim", "pcx_complex_copy_device", "pcx_backward",
    "pcx_extract_batch", "pcx_batch_info", "pcx_batch_copy", "pcx_batch_summary", "pcx_batch_free",
    "pcx_batch_tune", "pcx_server_create", "pcx_server_submit", "pcx_server_poll", "pcx_server_wait",
    "pcx_server_copy", "pcx_server_release", "pcx_server_stats", "pcx_server_destroy", "pcx_extract_into",
    "pcx_batch_steps",
]
PCX_F64, PCX_F32 = 0, 1


class PcxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pcx error {code}: {msg}")
        self.code = code


class _Opts(C.Structure):
    _fields_ = [("include_output", C.c_int32), ("timing", C.c_int32), ("pairing", C.c_int32),
                ("record_tape", C.c_int32), ("max_bytes", C.c_uint64), ("stream", C.c_void_p),
                ("batch_wg_per_cu", C.c_int32), ("prune", C.c_int32), ("verify_pairs", C.c_int32)]


class _BatchStats(C.Structure):
    _fields_ = [("n", C.c_int64), ("total_V", C.c_int64), ("total_E", C.c_int64), ("total_splits", C.c_int64),
                ("fallbacks", C.c_int32), ("degenerate", C.c_int32), ("workgroups", C.c_int32),
                ("wg_per_cu", C.c_int32), ("kernel_ms", C.c_double), ("time_ms", C.c_double),
                ("split_lanes", C.c_int32), ("select_items", C.c_int32)]


class _BatchTuning(C.Structure):
    _fields_ = [("wg_per_cu", C.c_int32), ("split_lanes", C.c_int32), ("select_items", C.c_int32),
                ("candidates", C.c_int32), ("ms_default", C.c_double), ("ms_best", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("V", C.c_int64), ("E", C.c_int64), ("D", C.c_int32), ("M", C.c_int32), ("Wd", C.c_int32),
                ("n_steps", C.c_int32), ("total_splits", C.c_int64), ("total_pairs", C.c_int64),
                ("peak_bytes", C.c_uint64), ("time_ms", C.c_double), ("exact_steps", C.c_int32),
                ("from_graph", C.c_int32)]


class _ServerOpts(C.Structure):
    _fields_ = [("mem_budget", C.c_uint64), ("max_batch", C.c_int32), ("large_workers", C.c_int32),
                ("include_output", C.c_int32), ("small_vertices", C.c_int32)]


class _ServerResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("batched", C.c_int32), ("V", C.c_int64), ("E", C.c_int64),
                ("total_splits", C.c_int64), ("latency_ms", C.c_double), ("queue_ms", C.c_double),
                ("D", C.c_int32), ("Wd", C.c_int32)]


class _ServerSummary(C.Structure):
    _fields_ = [("completed", C.c_int64), ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("p50_queue_ms", C.c_double), ("p99_queue_ms", C.c_double), ("span_s", C.c_double),
                ("jobs_per_s", C.c_double), ("splits_per_s", C.c_double), ("vertices_per_s", C.c_double),
                ("ticks", C.c_int64), ("mean_tick_jobs", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2306_07212_amd.build` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    PD = C.POINTER(C.c_double)
    lib.pcx_last_error.restype = C.c_char_p
    lib.pcx_mlp_create.argtypes = [i32, C.POINTER(i32), C.POINTER(PD), C.POINTER(PD), C.POINTER(vp)]
    lib.pcx_mlp_free.argtypes = [vp]
    lib.pcx_mlp_free.restype = None
    lib.pcx_extract.argtypes = [vp, PD, PD, C.POINTER(_Opts), C.POINTER(vp)]
    lib.pcx_extract_simplex.argtypes = [vp, PD, C.POINTER(_Opts), C.POINTER(vp)]
    lib.pcx_cell_counts.argtypes = [vp, C.POINTER(i64), vp]
    lib.pcx_regions.argtypes = [vp, vp, C.POINTER(i64), vp]
    lib.pcx_complex_info.argtypes = [vp, C.POINTER(_Info)]
    lib.pcx_complex_steps.argtypes = [vp, vp]
    lib.pcx_complex_copy.argtypes = [vp, vp, vp, vp]
    lib.pcx_complex_device.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
    lib.pcx_complex_kernel_time.argtypes = [vp, i32, PD, C.POINTER(i64)]
    lib.pcx_complex_free.argtypes = [vp]
    lib.pcx_complex_free.restype = None
    lib.pcx_complex_copy_device.argtypes = [vp, vp, vp, vp, vp]
    lib.pcx_backward.argtypes = [vp, vp, vp, C.POINTER(vp), C.POINTER(vp), i32, vp]
    lib.pcx_extract_batch.argtypes = [i32, C.POINTER(vp), PD, PD, C.POINTER(_Opts), C.POINTER(vp)]
    lib.pcx_batch_info.argtypes = [vp, i32, C.POINTER(_Info)]
    lib.pcx_batch_copy.argtypes = [vp, i32, vp, vp, vp]
    lib.pcx_batch_steps.argtypes = [vp, i32, vp]
    lib.pcx_batch_summary.argtypes = [vp, C.POINTER(_BatchStats)]
    lib.pcx_batch_free.argtypes = [vp]
    lib.pcx_batch_free.restype = None
    lib.pcx_batch_tune.argtypes = [i32, C.POINTER(vp), PD, PD, C.POINTER(_Opts), C.POINTER(_BatchTuning)]
    u64p = C.POINTER(C.c_uint64)
    lib.pcx_server_create.argtypes = [C.POINTER(_ServerOpts), C.POINTER(vp)]
    lib.pcx_server_submit.argtypes = [vp, vp, PD, PD, u64p]
    lib.pcx_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(_ServerResult)]
    lib.pcx_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(_ServerResult)]
    lib.pcx_server_copy.argtypes = [vp, C.c_uint64, vp, vp, vp]
    lib.pcx_server_release.argtypes = [vp, C.c_uint64]
    lib.pcx_server_stats.argtypes = [vp, C.POINTER(_ServerSummary)]
    lib.pcx_server_destroy.argtypes = [vp]
    lib.pcx_server_destroy.restype = None
    lib.pcx_extract_into.argtypes = [vp, PD, PD, C.POINTER(_Opts), vp, vp, vp, i64, i64, C.POINTER(_Info), vp]
    lib.pcx_cache_trim.argtypes = []
    lib.pcx_cache_trim.restype = None
    for s in SYMBOLS:
        getattr(lib, s)
    return lib


_lib = _load()


def _check(rc: int):
    if rc != PCX_OK:
        raise PcxError(rc, _lib.pcx_last_error().decode())


def cache_trim() -> None:
    """``pcx_cache_trim``: give cached device blocks back to the HIP runtime."""
    _lib.pcx_cache_trim()


def last_error() -> str:
    return _lib.pcx_last_error().decode()


class MLP:
    """A ReLU MLP on the device (``pcx_mlp_create``). W[l] is [N_l, N_{l-1}]."""

    def __init__(self, widths: Sequence[int], W, b):
        self.widths = [int(w) for w in widths]
        L = len(self.widths) - 1
        Wc = [np.ascontiguousarray(w, np.float64) for w in W]
        bc = [np.ascontiguousarray(x, np.float64) for x in b]
        if len(Wc) != L or len(bc) != L:
            raise ValueError("need one W and one b per layer")
        for l in range(L):
            if Wc[l].shape != (self.widths[l + 1], self.widths[l]) or bc[l].shape != (self.widths[l + 1],):
                raise ValueError(f"layer {l}: W must be [{self.widths[l + 1]}, {self.widths[l]}]")
        PD = C.POINTER(C.c_double)
        wa = (PD * L)(*[w.ctypes.data_as(PD) for w in Wc])
        ba = (PD * L)(*[x.ctypes.data_as(PD) for x in bc])
        ws = (C.c_int32 * (L + 1))(*self.widths)
        h = C.c_void_p()
        _check(_lib.pcx_mlp_create(L, ws, wa, ba, C.byref(h)))
        self._h = h

    @classmethod
    def from_net(cls, net) -> "MLP":
        return cls(net.widths, net.W, net.b)

    @property
    def D(self) -> int:
        return self.widths[0]

    def close(self):
        if getattr(self, "_h", None):
            _lib.pcx_mlp_free(self._h)
            self._h = None

    def __del__(self):
        # at interpreter exit the library handle (and the HIP runtime) may already be gone
        if _lib is not None and not sys.is_finalizing():
            self.close()


@dataclass
class Info:
    V: int
    E: int
    D: int
    M: int
    Wd: int
    n_steps: int
    total_splits: int
    total_pairs: int
    peak_bytes: int
    time_ms: float
    exact_steps: int = 0
    from_graph: int = 0


def sign_layout(widths: Sequence[int], include_output: bool = False, m: Optional[int] = None):
    """(word, shift) of every sign-vector entry under the packing of pcx.h: the
    m domain entries in word 0 (2D for the box, D+1 for a simplex), each
    subdivided layer from a fresh word."""
    D = int(widths[0])
    m = 2 * D if m is None else int(m)
    L = len(widths) - 1
    nsub = L if include_output else L - 1
    word = [0] * m
    shift = [2 * e for e in range(m)]
    lw = 1
    for l in range(1, nsub + 1):
        for i in range(int(widths[l])):
            word.append(lw + (i >> 5))
            shift.append(2 * (i & 31))
        lw += (int(widths[l]) + 31) // 32
    return np.array(word, np.int64), np.array(shift, np.int64), lw


class Complex:
    """An extracted 1-skeleton held on the device (``pcx_complex``)."""

    def __init__(self, handle, widths, include_output, m=None):
        self._h = handle
        self.widths = list(widths)
        self.include_output = include_output
        self.m = 2 * int(widths[0]) if m is None else int(m)  # domain entries

    def info(self) -> Info:
        i = _Info()
        _check(_lib.pcx_complex_info(self._h, C.byref(i)))
        return Info(i.V, i.E, i.D, i.M, i.Wd, i.n_steps, i.total_splits, i.total_pairs, i.peak_bytes, i.time_ms,
                    i.exact_steps, i.from_graph)

    def steps(self) -> np.ndarray:
        n = self.info().n_steps
        out = np.zeros((n, 4), np.int64)
        _check(_lib.pcx_complex_steps(self._h, out.ctypes.data))
        return out

    def copy(self):
        """(coords [V, D] float64, packed signs [V, Wd] uint64, edges [E, 2] int32) on the host."""
        inf = self.info()
        X = np.empty((inf.V, inf.D), np.float64)
        SG = np.empty((inf.V, inf.Wd), np.uint64)
        Ed = np.empty((inf.E, 2), np.int32)
        _check(_lib.pcx_complex_copy(self._h, X.ctypes.data, SG.ctypes.data, Ed.ctypes.data))
        return X, SG, Ed

    def signs(self, packed: Optional[np.ndarray] = None) -> np.ndarray:
        """Sign-vectors as int8 [V, M] in {+1, 0, -1}."""
        if packed is None:
            _, packed, _ = self.copy()
        word, shift, _ = sign_layout(self.widths, self.include_output, self.m)
        codes = (packed[:, word] >> shift.astype(np.uint64)) & np.uint64(3)
        out = np.zeros(codes.shape, np.int8)
        out[codes == 1] = 1
        out[codes == 2] = -1
        return out

    def cell_counts(self, stream=None) -> np.ndarray:
        """``pcx_cell_counts``: the f-vector (f_0 = V, f_1 = E, ..., f_D = regions)."""
        D = self.info().D
        out = np.zeros(D + 1, np.int64)
        _check(_lib.pcx_cell_counts(self._h, out.ctypes.data_as(C.POINTER(C.c_int64)), stream))
        return out

    def regions(self, stream=None) -> np.ndarray:
        """``pcx_regions``: packed sign rows of every region, sorted ([n, Wd] uint64)."""
        n = C.c_int64()
        _check(_lib.pcx_regions(self._h, None, C.byref(n), stream))
        out = np.zeros((n.value, self.info().Wd), np.uint64)
        if n.value:
            _check(_lib.pcx_regions(self._h, out.ctypes.data, C.byref(n), stream))
        return out

    def copy_device(self, coords_ptr=None, signs_ptr=None, edges_ptr=None, stream=None):
        """``pcx_complex_copy_device`` into caller-owned device buffers (raw pointers)."""
        _check(_lib.pcx_complex_copy_device(self._h, coords_ptr, signs_ptr, edges_ptr, stream))

    def device_pointers(self):
        a, b, c = C.c_void_p(), C.c_void_p(), C.c_void_p()
        _check(_lib.pcx_complex_device(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def kernel_time(self, family: str):
        ms, n = C.c_double(), C.c_int64()
        _check(_lib.pcx_complex_kernel_time(self._h, KERNEL_FAMILIES.index(family), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.pcx_complex_free(self._h)
            self._h = None

    def __del__(self):
        # at interpreter exit the library handle (and the HIP runtime) may already be gone
        if _lib is not None and not sys.is_finalizing():
            self.close()


def timing_mask(families) -> int:
    """Bitmask for ``extract(timing=...)`` from family names (or True for all)."""
    if families is True:
        return (1 << len(KERNEL_FAMILIES)) - 1
    if not families:
        return 0
    return sum(1 << KERNEL_FAMILIES.index(f) for f in families)


def backward(mlp: MLP, cx: Complex, grad_coords_ptr: int, gW_ptrs, gb_ptrs, precision: int = PCX_F64,
             stream=None) -> None:
    """``pcx_backward``: dL/dW, dL/db (device buffers, overwritten) from dL/dx (device pointer)."""
    L = len(mlp.widths) - 1
    gw = (C.c_void_p * L)(*[int(p) for p in gW_ptrs])
    gb = (C.c_void_p * L)(*[int(p) for p in gb_ptrs])
    _check(_lib.pcx_backward(mlp._h, cx._h, grad_coords_ptr, gw, gb, int(precision), stream))


def extract(mlp: MLP, lo, hi, include_output: bool = False, timing=0, stream=None,
            max_bytes: int = 0, pairing: str = "hash", record_tape: bool = False, prune: bool = False,
            verify_pairs: bool = False) -> Complex:
    """``pcx_extract``: edge subdivision of the box [lo, hi] by every subdivided neuron.
    ``prune`` (with ``include_output``): pruning during subdivision for the output's level set.
    ``verify_pairs``: compare the perturbed sign rows of every hash-table pair too."""
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    if lo.shape != (mlp.D,) or hi.shape != (mlp.D,):
        raise ValueError("lo and hi must have D entries")
    tm = timing if isinstance(timing, int) and not isinstance(timing, bool) else timing_mask(timing)
    o = _Opts(int(bool(include_output)), int(tm), PAIRING[pairing], int(bool(record_tape)), int(max_bytes), stream, 0,
              int(bool(prune)), int(bool(verify_pairs)))
    h = C.c_void_p()
    PD = C.POINTER(C.c_double)
    _check(_lib.pcx_extract(mlp._h, lo.ctypes.data_as(PD), hi.ctypes.data_as(PD), C.byref(o), C.byref(h)))
    return Complex(h, mlp.widths, include_output)


def extract_into(mlp: MLP, lo, hi, coords_ptr: int, signs_ptr: int, edges_ptr: int, max_vertices: int,
                 max_edges: int, include_output: bool = False, stream=None, verify_pairs: bool = False):
    """``pcx_extract_into``: the extraction written into caller-allocated device
    buffers (raw pointers), with no device allocation by the library. Returns
    (Info, per-step counters [n_steps, 4] int64)."""
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    if lo.shape != (mlp.D,) or hi.shape != (mlp.D,):
        raise ValueError("lo and hi must have D entries")
    o = _Opts(int(bool(include_output)), 0, 0, 0, 0, stream, 0, 0, int(bool(verify_pairs)))
    L = len(mlp.widths) - 1
    n_steps = sum(mlp.widths[1:L + 1 if include_output else L])
    steps = np.zeros((max(1, n_steps), 4), np.int64)
    i = _Info()
    PD = C.POINTER(C.c_double)
    _check(_lib.pcx_extract_into(mlp._h, lo.ctypes.data_as(PD), hi.ctypes.data_as(PD), C.byref(o), coords_ptr,
                                 signs_ptr, edges_ptr, int(max_vertices), int(max_edges), C.byref(i),
                                 steps.ctypes.data))
    info = Info(i.V, i.E, i.D, i.M, i.Wd, i.n_steps, i.total_splits, i.total_pairs, i.peak_bytes, i.time_ms,
                i.exact_steps)
    return info, steps[:n_steps]


def extract_simplex(mlp: MLP, corners, include_output: bool = False, timing=0, stream=None, max_bytes: int = 0,
                    pairing: str = "hash", record_tape: bool = False, prune: bool = False,
                    verify_pairs: bool = False) -> Complex:
    """``pcx_extract_simplex``: edge subdivision of the simplex with the given D + 1
    corners (rows); sign entries 0..D are the barycentric coordinates."""
    P = np.ascontiguousarray(corners, np.float64)
    if P.shape != (mlp.D + 1, mlp.D):
        raise ValueError("corners must be (D + 1) x D")
    tm = timing if isinstance(timing, int) and not isinstance(timing, bool) else timing_mask(timing)
    o = _Opts(int(bool(include_output)), int(tm), PAIRING[pairing], int(bool(record_tape)), int(max_bytes), stream, 0,
              int(bool(prune)), int(bool(verify_pairs)))
    h = C.c_void_p()
    PD = C.POINTER(C.c_double)
    _check(_lib.pcx_extract_simplex(mlp._h, P.ctypes.data_as(PD), C.byref(o), C.byref(h)))
    return Complex(h, mlp.widths, include_output, m=mlp.D + 1)


@dataclass
class BatchStats:
    n: int
    total_V: int
    total_E: int
    total_splits: int
    fallbacks: int
    degenerate: int
    workgroups: int
    wg_per_cu: int
    kernel_ms: float
    time_ms: float
    split_lanes: int = 32
    select_items: int = 16


def _batch_args(mlps, boxes):
    arr = (C.c_void_p * len(mlps))(*[m._h.value for m in mlps])
    lo = np.ascontiguousarray(np.concatenate([np.asarray(b[0], np.float64) for b in boxes]) if boxes else np.zeros(1))
    hi = np.ascontiguousarray(np.concatenate([np.asarray(b[1], np.float64) for b in boxes]) if boxes else np.zeros(1))
    return arr, lo, hi


class Batch:
    """``pcx_extract_batch``: many networks in one persistent launch."""

    def __init__(self, mlps, boxes, include_output: bool = False, wg_per_cu: int = 0, stream=None,
                 max_bytes: int = 0, verify_pairs: bool = False):
        self.mlps = list(mlps)
        self.include_output = include_output
        arr, lo, hi = _batch_args(self.mlps, boxes)
        PD = C.POINTER(C.c_double)
        o = _Opts(int(bool(include_output)), 0, 0, 0, int(max_bytes), stream, int(wg_per_cu), 0,
                  int(bool(verify_pairs)))
        h = C.c_void_p()
        _check(_lib.pcx_extract_batch(len(self.mlps), arr, lo.ctypes.data_as(PD), hi.ctypes.data_as(PD),
                                      C.byref(o), C.byref(h)))
        self._h = h

    def __len__(self):
        return len(self.mlps)

    def info(self, i) -> Info:
        x = _Info()
        _check(_lib.pcx_batch_info(self._h, int(i), C.byref(x)))
        return Info(x.V, x.E, x.D, x.M, x.Wd, x.n_steps, x.total_splits, x.total_pairs, x.peak_bytes, x.time_ms)

    def copy(self, i):
        inf = self.info(i)
        X = np.empty((inf.V, inf.D), np.float64)
        SG = np.empty((inf.V, inf.Wd), np.uint64)
        Ed = np.empty((inf.E, 2), np.int32)
        _check(_lib.pcx_batch_copy(self._h, int(i), X.ctypes.data, SG.ctypes.data, Ed.ctypes.data))
        return X, SG, Ed

    def steps(self, i) -> np.ndarray:
        """Per-step counters of network i ([n_steps, 4] int64, as Complex.steps)."""
        out = np.zeros((self.info(i).n_steps, 4), np.int64)
        _check(_lib.pcx_batch_steps(self._h, int(i), out.ctypes.data))
        return out

    def stats(self) -> BatchStats:
        x = _BatchStats()
        _check(_lib.pcx_batch_summary(self._h, C.byref(x)))
        return BatchStats(x.n, x.total_V, x.total_E, x.total_splits, x.fallbacks, x.degenerate, x.workgroups,
                          x.wg_per_cu, x.kernel_ms, x.time_ms, x.split_lanes, x.select_items)

    def close(self):
        if getattr(self, "_h", None):
            _lib.pcx_batch_free(self._h)
            self._h = None

    def __del__(self):
        # at interpreter exit the library handle (and the HIP runtime) may already be gone
        if _lib is not None and not sys.is_finalizing():
            self.close()


def batch_tune(mlps, boxes, include_output: bool = False) -> dict:
    """``pcx_batch_tune``: the schedule and occupancy chosen for this batch's
    size signature (and the kernel times with the default and chosen ones)."""
    arr, lo, hi = _batch_args(list(mlps), boxes)
    PD = C.POINTER(C.c_double)
    o = _Opts(int(bool(include_output)), 0, 0, 0, 0, None, 0, 0)
    r = _BatchTuning()
    _check(_lib.pcx_batch_tune(len(mlps), arr, lo.ctypes.data_as(PD), hi.ctypes.data_as(PD), C.byref(o),
                               C.byref(r)))
    return _as_dict(r)


def _as_dict(st):
    return {k: getattr(st, k) for k, _ in st._fields_}


class Server:
    """``pcx_server_*``: continuous batching of extraction requests."""

    def __init__(self, mem_budget: int = 0, max_batch: int = 0, large_workers: int = 0,
                 include_output: bool = False, small_vertices: int = 0):
        o = _ServerOpts(int(mem_budget), int(max_batch), int(large_workers), int(bool(include_output)),
                        int(small_vertices))
        h = C.c_void_p()
        _check(_lib.pcx_server_create(C.byref(o), C.byref(h)))
        self._h = h
        self._keep = {}  # ticket -> (mlp, lo, hi): handles stay alive until release

    def submit(self, mlp: MLP, lo, hi) -> int:
        lo = np.ascontiguousarray(lo, np.float64)
        hi = np.ascontiguousarray(hi, np.float64)
        PD = C.POINTER(C.c_double)
        t = C.c_uint64()
        _check(_lib.pcx_server_submit(self._h, mlp._h, lo.ctypes.data_as(PD), hi.ctypes.data_as(PD), C.byref(t)))
        self._keep[t.value] = (mlp, lo, hi)
        return t.value

    def poll(self, ticket: int):
        r = _ServerResult()
        rc = _lib.pcx_server_poll(self._h, C.c_uint64(ticket), C.byref(r))
        if rc == PCX_PENDING:
            return None
        _check(rc)
        return _as_dict(r)

    def wait(self, ticket: int):
        r = _ServerResult()
        _check(_lib.pcx_server_wait(self._h, C.c_uint64(ticket), C.byref(r)))
        return _as_dict(r)

    def error(self, ticket: int) -> str:
        """The failure message of a finished request ("" if it succeeded)."""
        r = self.wait(ticket)
        if r["status"] == PCX_OK:
            return ""
        _lib.pcx_server_copy(self._h, C.c_uint64(ticket), None, None, None)
        return _lib.pcx_last_error().decode()

    def copy(self, ticket: int):
        r = self.wait(ticket)
        if r["status"] != PCX_OK:
            raise PcxError(r["status"], self.error(ticket))
        # row sizes as the server reports them (the output word is counted with include_output)
        D, Wd = r["D"], r["Wd"]
        X = np.empty((r["V"], D), np.float64)
        SG = np.empty((r["V"], Wd), np.uint64)
        Ed = np.empty((r["E"], 2), np.int32)
        _check(_lib.pcx_server_copy(self._h, C.c_uint64(ticket), X.ctypes.data, SG.ctypes.data, Ed.ctypes.data))
        return X, SG, Ed

    def release(self, ticket: int):
        _check(_lib.pcx_server_release(self._h, C.c_uint64(ticket)))
        self._keep.pop(ticket, None)

    def stats(self):
        st = _ServerSummary()
        _check(_lib.pcx_server_stats(self._h, C.byref(st)))
        return _as_dict(st)

    def close(self):
        if getattr(self, "_h", None):
            _lib.pcx_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        # at interpreter exit the library handle (and the HIP runtime) may already be gone
        if _lib is not None and not sys.is_finalizing():
            self.close()
