"""CPU oracle for the two-source FCA EM -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package. The product path (the HIP
library and its Python binding) never imports it, and the two share no code.

``fca_oracle.c`` is a plain FP64 C implementation of the conventional EM of
Section 2 of the FastFCA paper (likelihood eq. like, E-step eqs. MMSE and
postquadexp, M-step eqs. vupdate and Supdate). This module compiles it with
gcc and wraps it with ctypes. Arrays use y[f, n, m], S[j, f, m, m'],
v[j, f, n], x[j, f, n, m].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fca_oracle.c")
_LIB = os.path.join(_HERE, "libfca_oracle.so")

FLAG_NOT_PD = 1
FLAG_NONFINITE = 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                        "-shared", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i = ctypes.c_int
        lib.fca_oracle_em.argtypes = [i, i, i, dp, dp, dp, i, i, dp, dp, dp, ip]
        lib.fca_oracle_mmse.argtypes = [i, i, i, dp, dp, dp, i, dp]
        lib.fca_oracle_loglik.argtypes = [i, i, i, dp, dp, dp, i, dp]
        lib.fca_oracle_default_init.argtypes = [i, i, i, dp, dp, dp]
        for fn in (lib.fca_oracle_em, lib.fca_oracle_mmse, lib.fca_oracle_loglik,
                   lib.fca_oracle_default_init):
            fn.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_init(y: np.ndarray):
    """(S0 [2,F,M,M], v0 [2,F,N]) of the plain start (R1 = I,
    R2 = I + 0.5 e1 e1^H, v_j = ||y||^2 / M floored)."""
    y = _c128(y)
    F, N, M = y.shape
    S0 = np.zeros((2, F, M, M), np.complex128)
    v0 = np.zeros((2, F, N), np.float64)
    rc = _load().fca_oracle_default_init(M, F, N, _dp(y), _dp(S0), _dp(v0))
    if rc:
        raise ValueError("fca_oracle_default_init: invalid sizes")
    return S0, v0


def em(y: np.ndarray, S0: np.ndarray, v0: np.ndarray, iters: int, threads: int = 0):
    """Run ``iters`` conventional EM iterations.

    Returns (S [2,F,M,M], v [2,F,N], ll [iters+1, F], flags [F]) where
    ll[l, f] is the log-likelihood of theta^(l) at frequency f."""
    y = _c128(y)
    F, N, M = y.shape
    S0 = _c128(S0)
    v0 = _f64(v0)
    assert S0.shape == (2, F, M, M) and v0.shape == (2, F, N)
    S = np.zeros_like(S0)
    v = np.zeros_like(v0)
    ll = np.zeros((iters + 1, F), np.float64)
    flags = np.zeros(F, np.int32)
    rc = _load().fca_oracle_em(M, F, N, _dp(y), _dp(S0), _dp(v0), iters, threads, _dp(S),
                               _dp(v), _dp(ll), flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if rc:
        raise ValueError("fca_oracle_em: invalid sizes")
    return S, v, ll, flags


def mmse(y: np.ndarray, S: np.ndarray, v: np.ndarray, threads: int = 0) -> np.ndarray:
    """MMSE source images x[2,F,N,M] under (S, v), eq. (MMSE)."""
    y = _c128(y)
    F, N, M = y.shape
    x = np.zeros((2, F, N, M), np.complex128)
    rc = _load().fca_oracle_mmse(M, F, N, _dp(y), _dp(_c128(S)), _dp(_f64(v)), threads, _dp(x))
    if rc < 0:
        raise ValueError("fca_oracle_mmse: invalid sizes")
    return x


def loglik(y: np.ndarray, S: np.ndarray, v: np.ndarray, threads: int = 0) -> np.ndarray:
    """Per-frequency log-likelihood [F] of (S, v) under eq. (like)."""
    y = _c128(y)
    F, N, M = y.shape
    ll = np.zeros(F, np.float64)
    rc = _load().fca_oracle_loglik(M, F, N, _dp(y), _dp(_c128(S)), _dp(_f64(v)), threads, _dp(ll))
    if rc:
        raise ValueError("fca_oracle_loglik: invalid sizes")
    return ll
