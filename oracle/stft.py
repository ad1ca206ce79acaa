"""STFT analysis and overlap-add synthesis -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module; the product path never does.

The experiments of Section 4 (Table 1) analyse 16 kHz recordings with frames
of 1024 samples, a frame shift of 512 samples and a square-root Hann window,
and resynthesise the separated images the same way. Written out here from
the definitions, in FP64, for frame length L (a power of two) and shift
S = L / 2:

  window     w(t) = sin(pi t / L), t = 0 .. L-1  (the square root of the
             periodic Hann window 0.5 - 0.5 cos(2 pi t / L)); at 50 %
             overlap w(t)^2 + w(t + S)^2 = 1, so analysis and synthesis
             with the same window reconstruct the signal exactly.
  framing    frame n (n = 0 .. N-1) holds samples n S - S + t, t = 0 .. L-1
             (zero outside 0 .. T-1), N = floor((T - 1) / S) + 2, so every
             sample lies in two frames.
  analysis   X[f, n, m] = sum_t w(t) x_m(n S - S + t) exp(-2 pi i f t / L),
             f = 0 .. L/2 (the DFT, by its defining sum).
  synthesis  each frame's inverse DFT over the Hermitian extension
             (X[L - k] = conj X[k] for 0 < k < L/2; the real part taken),
             windowed by w and overlap-added at its frame position.

Layouts: x [M, T] real, X [F, N, M] complex (F = L/2 + 1; the layout the
EM takes as its mixture y(n, f)).
"""
from __future__ import annotations

import numpy as np


def window(L: int) -> np.ndarray:
    t = np.arange(L)
    return np.sin(np.pi * t / L)


def frames(T: int, L: int) -> int:
    S = L // 2
    return (T - 1) // S + 2


def dft_matrix(L: int) -> np.ndarray:
    """[L, L] with entry (k, t) = exp(-2 pi i k t / L)."""
    k = np.arange(L)
    return np.exp(-2j * np.pi * np.outer(k, k) / L)


def stft(x: np.ndarray, L: int) -> np.ndarray:
    """X [F, N, M] of the real signals x [M, T]."""
    x = np.asarray(x, dtype=np.float64)
    M, T = x.shape
    S, F, N = L // 2, L // 2 + 1, frames(T, L)
    w = window(L)
    D = dft_matrix(L)[:F]                        # rows f = 0 .. L/2
    X = np.zeros((F, N, M), dtype=np.complex128)
    for m in range(M):
        for n in range(N):
            seg = np.zeros(L)
            for t in range(L):
                s = n * S - S + t
                if 0 <= s < T:
                    seg[t] = x[m, s]
            X[:, n, m] = D @ (w * seg)
    return X


def istft(X: np.ndarray, T: int, L: int) -> np.ndarray:
    """x [M, T] from X [F, N, M] by windowed overlap-add of the frames'
    inverse DFTs (real part)."""
    X = np.asarray(X, dtype=np.complex128)
    F, N, M = X.shape
    S = L // 2
    assert F == L // 2 + 1 and N == frames(T, L)
    w = window(L)
    Dinv = np.conj(dft_matrix(L)) / L            # inverse DFT
    x = np.zeros((M, T))
    for m in range(M):
        for n in range(N):
            full = np.zeros(L, dtype=np.complex128)
            full[:F] = X[:, n, m]
            for k in range(F, L):
                full[k] = np.conj(X[L - k, n, m])
            seg = (Dinv @ full).real * w
            for t in range(L):
                s = n * S - S + t
                if 0 <= s < T:
                    x[m, s] += seg[t]
    return x
