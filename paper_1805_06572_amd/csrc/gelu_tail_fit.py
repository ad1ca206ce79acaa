"""Fit of the polynomial GELU used by the MLP kernels (fca_mlp.hip).

GELU(x) = x Phi(x) = max(x, 0) - t Phi(-t), t = |x|. The even tail
t Phi(-t) is approximated by t P(t) with P of degree 6 on [0, T], T = 4,
and t is clamped to T beyond it (the tail is 1.3e-4 there). The fit is a
weighted least-squares fit of t P(t) on a dense grid whose weights are
raised where the residual is large (iteratively reweighted, which drives it
towards equal ripple). Run it to print the coefficients (FP32, low order
first) and the worst error on the whole line with FP32 Horner evaluation.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erfc

T, DEG = 4.0, 6


def fit(T: float = T, deg: int = DEG, rounds: int = 60) -> np.ndarray:
    t = np.linspace(0.0, T, 40001)
    tail = t * 0.5 * erfc(t / np.sqrt(2.0))
    V = np.vander(t, deg + 1, increasing=True) * t[:, None]
    w = np.ones_like(t)
    for _ in range(rounds):
        c, *_ = np.linalg.lstsq(V * w[:, None], tail * w, rcond=None)
        e = V @ c - tail
        w = w * (1.0 + 3.0 * np.abs(e) / np.abs(e).max())
        w /= w.mean()
    return c.astype(np.float32)


def gelu_poly_f32(x: np.ndarray, c: np.ndarray, T: float = T) -> np.ndarray:
    """The kernel's evaluation order in FP32."""
    x = np.asarray(x, dtype=np.float32)
    t = np.minimum(np.abs(x), np.float32(T))
    p = np.full_like(t, c[-1])
    for k in range(len(c) - 2, -1, -1):
        p = (p * t + c[k]).astype(np.float32)
    return (np.maximum(x, np.float32(0)) - t * p).astype(np.float32)


if __name__ == "__main__":
    c = fit()
    x = np.linspace(-12.0, 12.0, 400001)
    err = np.abs(gelu_poly_f32(x, c).astype(np.float64) - x * 0.5 * erfc(-x / np.sqrt(2.0))).max()
    print("coefficients:", [float(v) for v in c])
    print(f"max |error| on [-12, 12]: {err:.3e}")
