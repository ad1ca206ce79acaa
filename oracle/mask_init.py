"""Mask-based initial spatial covariances -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module; the product path never does.

Section 4 of the FastFCA paper starts the EM from spatial covariances
estimated with time-frequency masks and gives no formula. The reading taken
here is the plain mask-weighted covariance, normalised to trace M and loaded
on the diagonal: with the powers v_j(n,f) of a start, r = v1 / (v1 + v2)
(1/2 where both are 0), sharpened to r^p / (r^p + (1 - r)^p), masks
w_1 = r and w_2 = 1 - r,

    A_j(f) = sum_n w_j(n,f) y(n,f) y(n,f)^H,
    R_j(f) = M A_j(f) / tr A_j(f) + load I     ((1 + load) I if tr A_j = 0).

Written out with explicit loops over frames in FP64, for checking by eye.
"""
from __future__ import annotations

import numpy as np


def masks(v0: np.ndarray, sharpen: float) -> np.ndarray:
    """[2, F, N] masks (w_1, w_2) from powers v0 [2, F, N]."""
    v = np.asarray(v0, dtype=np.float64)
    tot = v[0] + v[1]
    r = np.where(tot > 0, v[0] / np.where(tot > 0, tot, 1.0), 0.5)
    if sharpen != 1.0:
        a, b = r ** sharpen, (1.0 - r) ** sharpen
        r = a / (a + b)
    return np.stack([r, 1.0 - r])


def mask_covariances(y: np.ndarray, v0: np.ndarray, sharpen: float = 3.0, load: float = 1e-3) -> np.ndarray:
    """R [2, F, M, M] complex128 from y [F, N, M] and powers v0 [2, F, N]."""
    y = np.asarray(y, dtype=np.complex128)
    F, N, M = y.shape
    w = masks(v0, sharpen)
    R = np.zeros((2, F, M, M), dtype=np.complex128)
    for j in range(2):
        for f in range(F):
            A = np.zeros((M, M), dtype=np.complex128)
            for n in range(N):
                A += w[j, f, n] * np.outer(y[f, n], y[f, n].conj())
            tr = np.trace(A).real
            R[j, f] = M * A / tr if tr > 0 else np.eye(M)
            R[j, f] += load * np.eye(M)
    return R
