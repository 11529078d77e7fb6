"""FP64 CPU oracle for the PLUGIN bandwidth selector (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg use this package.  It loads ``liboracle.so`` built from
``oracle.c`` (plain C + OpenMP, FP64) and never touches the HIP library.

Every function follows Section 3 / Algorithm 1 of the paper; see the header of
``oracle.c`` for the step-by-step mapping and the readings taken where the
paper is silent.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK = 0
EINVAL = -1
ENONFINITE = -2
EDEGENERATE = -3
ENOMEM = -4


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with oracle status {code}")
        self.code = code


class _Result(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("mean", "sigma", "psi8", "g1", "psi6", "g2", "psi4", "h")]


@dataclass
class PluginResult:
    mean: float
    sigma: float
    psi8: float
    g1: float
    psi6: float
    g2: float
    psi4: float
    h: float


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        D, I64, I = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        PD = ctypes.POINTER(ctypes.c_double)
        lib.oracle_K6.argtypes = [D]; lib.oracle_K6.restype = D
        lib.oracle_K4.argtypes = [D]; lib.oracle_K4.restype = D
        lib.oracle_phi_deriv.argtypes = [I, D]; lib.oracle_phi_deriv.restype = D
        lib.oracle_moments.argtypes = [PD, I64, PD, PD]; lib.oracle_moments.restype = I
        lib.oracle_block_sum.argtypes = [PD, I64, I, D, I64, I64, I64, I64, PD]
        lib.oracle_block_sum.restype = I
        lib.oracle_pair_sum.argtypes = [PD, I64, I, D, PD]; lib.oracle_pair_sum.restype = I
        lib.oracle_psi.argtypes = [PD, I64, I, D, PD]; lib.oracle_psi.restype = I
        lib.oracle_plugin.argtypes = [PD, I64, ctypes.POINTER(_Result)]
        lib.oracle_plugin.restype = I
        lib.oracle_plugin_zscore.argtypes = [PD, I64, ctypes.POINTER(_Result)]
        lib.oracle_plugin_zscore.restype = I
        lib.oracle_kde_eval.argtypes = [PD, I64, D, PD, I64, PD]
        lib.oracle_kde_eval.restype = I
        lib.oracle_num_threads.argtypes = []; lib.oracle_num_threads.restype = I
        lib.oracle_set_num_threads.argtypes = [I]; lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def K6(u: float) -> float:
    return _load().oracle_K6(float(u))


def K4(u: float) -> float:
    return _load().oracle_K4(float(u))


def phi_deriv(r: int, u: float) -> float:
    return _load().oracle_phi_deriv(int(r), float(u))


def moments(x):
    a = _arr(x)
    m, s = ctypes.c_double(), ctypes.c_double()
    st = _load().oracle_moments(_ptr(a), a.size, ctypes.byref(m), ctypes.byref(s))
    if st:
        raise OracleError(st, "oracle_moments")
    return m.value, s.value


def block_sum(x, r: int, g: float, r0: int, r1: int, c0: int, c1: int) -> float:
    a = _arr(x)
    out = ctypes.c_double()
    st = _load().oracle_block_sum(_ptr(a), a.size, int(r), float(g), int(r0), int(r1),
                                  int(c0), int(c1), ctypes.byref(out))
    if st:
        raise OracleError(st, "oracle_block_sum")
    return out.value


def pair_sum(x, r: int, g: float) -> float:
    a = _arr(x)
    out = ctypes.c_double()
    st = _load().oracle_pair_sum(_ptr(a), a.size, int(r), float(g), ctypes.byref(out))
    if st:
        raise OracleError(st, "oracle_pair_sum")
    return out.value


def psi(x, r: int, g: float) -> float:
    a = _arr(x)
    out = ctypes.c_double()
    st = _load().oracle_psi(_ptr(a), a.size, int(r), float(g), ctypes.byref(out))
    if st:
        raise OracleError(st, "oracle_psi")
    return out.value


def _plugin(fn, x) -> PluginResult:
    a = _arr(x)
    res = _Result()
    st = fn(_ptr(a), a.size, ctypes.byref(res))
    if st:
        raise OracleError(st, "oracle_plugin")
    return PluginResult(*(getattr(res, k) for k, _ in _Result._fields_))


def plugin(x) -> PluginResult:
    return _plugin(_load().oracle_plugin, x)


def plugin_zscore(x) -> PluginResult:
    return _plugin(_load().oracle_plugin_zscore, x)


def kde_eval(x, h: float, pts) -> np.ndarray:
    a, p = _arr(x), _arr(pts)
    out = np.empty(p.size, dtype=np.float64)
    st = _load().oracle_kde_eval(_ptr(a), a.size, float(h), _ptr(p), p.size, _ptr(out))
    if st:
        raise OracleError(st, "oracle_kde_eval")
    return out


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(t: int) -> None:
    _load().oracle_set_num_threads(int(t))
