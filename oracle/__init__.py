"""Python binding of the oracle (test infrastructure only).

The oracle is a plain, slow FP64 (and long double) CPU implementation of the
tree-level |M|^2 that the GPU library computes: explicit Feynman diagrams with
explicit Dirac matrices, explicit SU(3) colour matrices, an explicit helicity
sum, plus the Philox4x32-10 generator and RAMBO phase space.  Only tests, the
smoke check and the CPU-baseline leg of the benchmark may import it; it shares
no code with the GPU path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["oracle.cpp", "oracle.h", "process.hpp", "lorentz.hpp", "colour.hpp", "philox_rambo.hpp", "events.hpp"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
               os.path.join(_HERE, "oracle.cpp"), "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("alpha_s", ctypes.c_double), ("alpha_em", ctypes.c_double),
                ("sin2w", ctypes.c_double), ("mz", ctypes.c_double), ("wz", ctypes.c_double),
                ("mt", ctypes.c_double), ("wt", ctypes.c_double), ("z_enabled", ctypes.c_int)]


_lib = None


def _stale() -> bool:
    if not os.path.exists(_LIB_PATH):
        return True
    t = os.path.getmtime(_LIB_PATH)
    return any(os.path.getmtime(os.path.join(_HERE, f)) > t for f in _SOURCES)


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.oracle_uniform_pair.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, dp]
        L.oracle_rambo.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_uint64,
                                   ctypes.c_uint64, ctypes.c_int64, dp, dp]
        L.oracle_external.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_process_new.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(_Params)]
        L.oracle_process_new.restype = ctypes.c_void_p
        L.oracle_process_free.argtypes = [ctypes.c_void_p]
        L.oracle_last_error.restype = ctypes.c_char_p
        L.oracle_process_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong)]
        L.oracle_colour_matrix.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong),
                                           ctypes.POINTER(ctypes.c_int)]
        L.oracle_me.argtypes = [ctypes.c_void_p, dp, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, dp]
        L.oracle_me_hel.argtypes = [ctypes.c_void_p, dp, ctypes.c_int, dp]
        L.oracle_condition.argtypes = [ctypes.c_void_p, dp, dp]
        L.oracle_gauge.argtypes = [ctypes.c_void_p, dp, ctypes.c_int, dp]
        L.oracle_flows.argtypes = [ctypes.c_void_p, dp, ctypes.c_int, dp]
        L.oracle_event_weights.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, dp, dp]
        L.oracle_unweight.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]
        L.oracle_unweight.restype = ctypes.c_int64
        L.oracle_select.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_int), dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# Standard-model parameters of the benchmark workloads.
DEFAULT_PARAMS = dict(alpha_s=0.118, alpha_em=1.0 / 132.5, sin2w=0.2222, mz=91.188, wz=2.441,
                      mt=173.0, wt=0.0, z_enabled=1)

PROCESSES = {
    "ee_mumu": [-11, 11, -13, 13],
    "gg_tt": [21, 21, 6, -6],
    "gg_ttg": [21, 21, 6, -6, 21],
    "gg_ttgg": [21, 21, 6, -6, 21, 21],
    "gg_ttggg": [21, 21, 6, -6, 21, 21, 21],
}


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def uniform_pair(seed: int, event: int, block: int):
    out = np.zeros(2)
    lib().oracle_uniform_pair(seed, event, block, _dp(out))
    return out


def rambo(masses_out, sqrt_s: float, seed: int, first_event: int, nevt: int):
    """Returns (mom [nevt][n_ext][4], wgt [nevt])."""
    m = np.ascontiguousarray(masses_out, dtype=np.float64)
    n_ext = len(m) + 2
    mom = np.zeros((nevt, n_ext, 4))
    wgt = np.zeros(nevt)
    rc = lib().oracle_rambo(len(m), _dp(m), sqrt_s, seed, first_event, nevt, _dp(mom), _dp(wgt))
    if rc != 0:
        raise ValueError("oracle_rambo failed")
    return mom, wgt


def event_weights(wgt, me, sqrt_s: float):
    """Cross-section weights in pb and (sum w, sum w^2, max w)."""
    wgt = np.ascontiguousarray(wgt, dtype=np.float64)
    me = np.ascontiguousarray(me, dtype=np.float64)
    w = np.zeros(len(wgt))
    st = np.zeros(3)
    if lib().oracle_event_weights(len(wgt), _dp(wgt), _dp(me), sqrt_s, _dp(w), _dp(st)) != 0:
        raise ValueError("oracle_event_weights failed")
    return w, st


def unweight(w, r, w_ref: float) -> np.ndarray:
    """Indices of the events kept by hit-or-miss against w_ref."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    idx = np.zeros(max(1, len(w)), dtype=np.int64)
    k = lib().oracle_unweight(len(w), _dp(w), _dp(r), w_ref, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return idx[:k].copy()


def external(kind: str, p, mass: float, hel: int) -> np.ndarray:
    kinds = {"u": 0, "v": 1, "ubar": 2, "vbar": 3, "eps": 4}
    pp = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(8)
    lib().oracle_external(kinds[kind], _dp(pp), mass, hel, _dp(out))
    return out[0::2] + 1j * out[1::2]


class Process:
    """An oracle process: plain Feynman-diagram |M|^2 on the CPU."""

    def __init__(self, pdg, **params):
        par = dict(DEFAULT_PARAMS)
        par.update(params)
        self.pdg = list(pdg)
        self.params = par
        arr = (ctypes.c_int * len(pdg))(*pdg)
        p = _Params(**par)
        h = lib().oracle_process_new(len(pdg), arr, ctypes.byref(p))
        if not h:
            raise ValueError(lib().oracle_last_error().decode())
        self._h = h
        info = (ctypes.c_longlong * 5)()
        lib().oracle_process_info(h, info)
        self.n_diagrams, self.n_terms, self.n_colour, self.n_hel, self.colour_den = [int(x) for x in info]
        self.n_ext = len(pdg)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_process_free(h)
            self._h = None

    def colour_matrix(self):
        """(numerators [ncol][ncol] int64, denominator, basis [ncol][k] legs)."""
        n = self.n_colour
        k = sum(1 for x in self.pdg if x == 21)
        num = (ctypes.c_longlong * (n * n))()
        basis = (ctypes.c_int * max(1, n * k))()
        lib().oracle_colour_matrix(self._h, num, basis)
        C = np.array(num[:], dtype=np.int64).reshape(n, n)
        B = np.array(basis[: n * k], dtype=np.int64).reshape(n, k)
        return C, self.colour_den, B

    def me(self, mom: np.ndarray, colour_mode: int = 0, precision: int = 0,
           nthreads: int = 1) -> np.ndarray:
        mom = np.ascontiguousarray(mom, dtype=np.float64)
        n = mom.shape[0]
        assert mom.shape[1:] == (self.n_ext, 4)
        out = np.zeros(n)
        rc = lib().oracle_me(self._h, _dp(mom), n, colour_mode, precision, nthreads, _dp(out))
        if rc != 0:
            raise ValueError(lib().oracle_last_error().decode())
        return out

    def me_hel(self, mom1: np.ndarray, precision: int = 0) -> np.ndarray:
        mom1 = np.ascontiguousarray(mom1, dtype=np.float64)
        out = np.zeros(self.n_hel)
        lib().oracle_me_hel(self._h, _dp(mom1), precision, _dp(out))
        return out

    def flows(self, mom1: np.ndarray, hel: int) -> np.ndarray:
        """Colour-ordered amplitudes of one helicity (basis order)."""
        mom1 = np.ascontiguousarray(mom1, dtype=np.float64)
        out = np.zeros(2 * self.n_colour)
        if lib().oracle_flows(self._h, _dp(mom1), hel, _dp(out)) != 0:
            raise ValueError("bad helicity")
        return out[0::2] + 1j * out[1::2]

    def select(self, mom1: np.ndarray, r_hel: float, r_col: float):
        """(helicity code, colour flow, margins) for one event."""
        mom1 = np.ascontiguousarray(mom1, dtype=np.float64)
        out = (ctypes.c_int * 2)()
        margin = np.zeros(2)
        lib().oracle_select(self._h, _dp(mom1), r_hel, r_col, out, _dp(margin))
        return int(out[0]), int(out[1]), margin

    def condition(self, mom1: np.ndarray) -> float:
        """Condition number of |M|^2 for one event (see oracle.h)."""
        mom1 = np.ascontiguousarray(mom1, dtype=np.float64)
        out = np.zeros(1)
        lib().oracle_condition(self._h, _dp(mom1), _dp(out))
        return float(out[0])

    def gauge(self, mom1: np.ndarray, leg: int):
        mom1 = np.ascontiguousarray(mom1, dtype=np.float64)
        out = np.zeros(2)
        rc = lib().oracle_gauge(self._h, _dp(mom1), leg, _dp(out))
        if rc != 0:
            raise ValueError("gauge test needs a gluon leg")
        return float(out[0]), float(out[1])
