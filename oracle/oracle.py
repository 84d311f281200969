"""ctypes front end of the C oracle (``pcx_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

``extract`` runs plain FP64 edge subdivision on the CPU (the steps of Sec. 4.2
of the paper, in order). ``forward`` is the plain forward pass of Sec. 3.4.
``vertex_solve`` recomputes one vertex from its sign-vector by solving the
D x D system of its zero entries.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcx_oracle.c")
_LIB = os.path.join(_HERE, "libpcx_oracle.so")
_lib = None

OK, ERR_INVALID, ERR_OOM, ERR_DEGENERATE, ERR_SINGULAR = 0, -1, -2, -3, -6


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc, FP64, no FMA contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Net(C.Structure):
    _fields_ = [("D", C.c_int), ("L", C.c_int), ("widths", C.POINTER(C.c_int)),
                ("W", C.POINTER(C.POINTER(C.c_double))), ("b", C.POINTER(C.POINTER(C.c_double)))]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(_LIB)
    vp = C.c_void_p
    lib.pcxo_extract.restype = vp
    lib.pcxo_extract.argtypes = [C.POINTER(_Net), C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int, C.c_int,
                                 C.c_int]
    lib.pcxo_extract_simplex.restype = vp
    lib.pcxo_extract_simplex.argtypes = [C.POINTER(_Net), C.POINTER(C.c_double), C.c_int, C.c_int, C.c_int]
    lib.pcxo_free.argtypes = [vp]
    lib.pcxo_set_threads.argtypes = [C.c_int]
    lib.pcxo_set_threads.restype = None
    for name, rt in [("pcxo_status", C.c_int), ("pcxo_V", C.c_long), ("pcxo_E", C.c_long),
                     ("pcxo_M", C.c_int), ("pcxo_n_steps", C.c_int), ("pcxo_min_margin", C.c_double)]:
        getattr(lib, name).restype = rt
        getattr(lib, name).argtypes = [vp]
    lib.pcxo_message.restype = C.c_char_p
    lib.pcxo_message.argtypes = [vp]
    lib.pcxo_copy.argtypes = [vp, vp, vp, vp, vp]
    lib.pcxo_forward.restype = C.c_int
    lib.pcxo_forward.argtypes = [C.POINTER(_Net), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.pcxo_vertex_solve.restype = C.c_int
    lib.pcxo_vertex_solve.argtypes = [C.POINTER(_Net), C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_int8), C.POINTER(C.c_double)]
    _lib = lib
    return lib


class _NetHolder:
    """Keeps the numpy buffers alive while the C struct points into them."""

    def __init__(self, widths: Sequence[int], W, b):
        self.widths = np.ascontiguousarray(widths, dtype=np.int32)
        self.W = [np.ascontiguousarray(w, dtype=np.float64) for w in W]
        self.b = [np.ascontiguousarray(x, dtype=np.float64) for x in b]
        L = len(self.W)
        assert len(self.widths) == L + 1
        for l in range(L):
            assert self.W[l].shape == (self.widths[l + 1], self.widths[l]), "W[l] must be [N_l][N_{l-1}]"
            assert self.b[l].shape == (self.widths[l + 1],)
        PD = C.POINTER(C.c_double)
        self._Wp = (PD * L)(*[w.ctypes.data_as(PD) for w in self.W])
        self._bp = (PD * L)(*[x.ctypes.data_as(PD) for x in self.b])
        self.c = _Net(int(self.widths[0]), L, self.widths.ctypes.data_as(C.POINTER(C.c_int)), self._Wp, self._bp)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class OracleResult:
    D: int
    M: int
    X: np.ndarray        # [V, D] float64
    S: np.ndarray        # [V, M] int8 in {+1, 0, -1}
    edges: np.ndarray    # [E, 2] int32
    steps: np.ndarray    # [n_steps, 4] int64: V_n, E_n, S_n, K_n
    min_margin: float

    @property
    def V(self):
        return self.X.shape[0]

    @property
    def E(self):
        return self.edges.shape[0]


def extract(net, lo, hi, include_output: bool = False, mutation: int = 0, prune: bool = False,
            threads: int = 1) -> OracleResult:
    """Edge subdivision of ``net`` on the box [lo, hi] (float64; the per-vertex
    loops on ``threads`` threads, one by default: the result does not depend on
    it). ``prune`` (with ``include_output``): drop, before each layer, the edges
    whose vertices agree on every neuron still to come (Sec. 5.4.2)."""
    lib = _load()
    h = _NetHolder(net.widths, net.W, net.b)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    lib.pcxo_set_threads(int(threads))
    try:
        r = lib.pcxo_extract(C.byref(h.c), _dp(lo), _dp(hi), int(bool(include_output)), int(bool(prune)),
                             int(mutation))
    finally:
        lib.pcxo_set_threads(1)
    if not r:
        raise MemoryError("oracle allocation failed")
    try:
        st = lib.pcxo_status(r)
        if st != OK:
            raise OracleError(st, lib.pcxo_message(r).decode())
        V, E, M, ns = lib.pcxo_V(r), lib.pcxo_E(r), lib.pcxo_M(r), lib.pcxo_n_steps(r)
        D = int(h.widths[0])
        X = np.empty((V, D), np.float64)
        S = np.empty((V, M), np.int8)
        Ed = np.empty((E, 2), np.int32)
        steps = np.empty((ns, 4), np.int64)
        lib.pcxo_copy(r, X.ctypes.data, S.ctypes.data, Ed.ctypes.data, steps.ctypes.data)
        return OracleResult(D, M, X, S, Ed, steps, float(lib.pcxo_min_margin(r)))
    finally:
        lib.pcxo_free(r)


def _result(lib, r, D) -> OracleResult:
    if not r:
        raise MemoryError("oracle allocation failed")
    try:
        st = lib.pcxo_status(r)
        if st != OK:
            raise OracleError(st, lib.pcxo_message(r).decode())
        V, E, M, ns = lib.pcxo_V(r), lib.pcxo_E(r), lib.pcxo_M(r), lib.pcxo_n_steps(r)
        X = np.empty((V, D), np.float64)
        S = np.empty((V, M), np.int8)
        Ed = np.empty((E, 2), np.int32)
        steps = np.empty((ns, 4), np.int64)
        lib.pcxo_copy(r, X.ctypes.data, S.ctypes.data, Ed.ctypes.data, steps.ctypes.data)
        return OracleResult(D, M, X, S, Ed, steps, float(lib.pcxo_min_margin(r)))
    finally:
        lib.pcxo_free(r)


def extract_simplex(net, corners, include_output: bool = False, mutation: int = 0,
                    prune: bool = False) -> OracleResult:
    """Edge subdivision on the simplex with the given D + 1 corners (rows); the
    first D + 1 sign-vector entries are the barycentric coordinates."""
    lib = _load()
    h = _NetHolder(net.widths, net.W, net.b)
    D = int(h.widths[0])
    P = np.ascontiguousarray(corners, dtype=np.float64)
    assert P.shape == (D + 1, D)
    r = lib.pcxo_extract_simplex(C.byref(h.c), _dp(P), int(bool(include_output)), int(bool(prune)), int(mutation))
    return _result(lib, r, D)


def forward(net, x) -> np.ndarray:
    """All pre-activations (layers 1..L concatenated) at each row of x: [n, sum N_l]."""
    lib = _load()
    h = _NetHolder(net.widths, net.W, net.b)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    tot = int(sum(h.widths[1:]))
    out = np.empty((x.shape[0], tot), np.float64)
    for i in range(x.shape[0]):
        st = lib.pcxo_forward(C.byref(h.c), _dp(x[i]), _dp(out[i]))
        if st != OK:
            raise OracleError(st, "forward")
    return out


def vertex_solve(net, lo, hi, sigma, include_output: bool = False) -> np.ndarray:
    """Coordinates of each vertex from its sign-vector (rows of ``sigma``, int8)."""
    lib = _load()
    h = _NetHolder(net.widths, net.W, net.b)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    sig = np.ascontiguousarray(np.atleast_2d(sigma), dtype=np.int8)
    D = int(h.widths[0])
    out = np.empty((sig.shape[0], D), np.float64)
    for i in range(sig.shape[0]):
        st = lib.pcxo_vertex_solve(C.byref(h.c), int(bool(include_output)), _dp(lo), _dp(hi),
                                   sig[i].ctypes.data_as(C.POINTER(C.c_int8)), _dp(out[i]))
        if st != OK:
            raise OracleError(st, f"vertex_solve row {i}")
    return out
