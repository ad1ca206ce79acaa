"""Pins of the STFT oracle (oracle/stft.py): a hand-worked tiny analysis,
numpy's FFT of the same windowed frames, perfect reconstruction, and the
window identities. CPU only."""
from __future__ import annotations

import json
import os

import numpy as np

from oracle import stft as ostft

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_worked_tiny_analysis_and_synthesis():
    g = json.load(open(os.path.join(GOLDEN, "stft_tiny.json")))
    L, x = g["L"], np.array([g["x"]])
    X = ostft.stft(x, L)
    r2 = np.sqrt(2.0)
    want = np.array([[complex(re[0] + re[1] * r2, im[0] + im[1] * r2) for re, im in frame]
                     for frame in g["X_frames_as_a_plus_b_sqrt2"]])      # [n][f]
    assert X.shape == (3, 3, 1)
    np.testing.assert_allclose(X[:, :, 0].T, want, rtol=0, atol=1e-14)
    np.testing.assert_allclose(ostft.istft(X, 3, L), x, rtol=0, atol=1e-14)


def test_analysis_equals_numpy_rfft_of_the_windowed_frames():
    rng = np.random.default_rng(0)
    L, T, M = 64, 301, 3
    x = rng.standard_normal((M, T))
    X = ostft.stft(x, L)
    S, w = L // 2, np.sin(np.pi * np.arange(L) / L)
    xp = np.concatenate([np.zeros((M, S)), x, np.zeros((M, L))], axis=1)
    for n in range(ostft.frames(T, L)):
        seg = xp[:, n * S:n * S + L] * w
        np.testing.assert_allclose(X[:, n, :], np.fft.rfft(seg, axis=1).T, rtol=0, atol=1e-12)


def test_perfect_reconstruction():
    rng = np.random.default_rng(1)
    for L, T in ((16, 1), (16, 8), (32, 100), (64, 257)):
        x = rng.standard_normal((2, T))
        np.testing.assert_allclose(ostft.istft(ostft.stft(x, L), T, L), x, rtol=0, atol=1e-12)


def test_window_is_root_hann_with_unit_overlap_sum():
    L = 1024
    w = ostft.window(L)
    t = np.arange(L)
    np.testing.assert_allclose(w ** 2, 0.5 - 0.5 * np.cos(2 * np.pi * t / L), atol=1e-15)
    np.testing.assert_allclose(w[:L // 2] ** 2 + w[L // 2:] ** 2, 1.0, atol=1e-15)
    assert ostft.frames(16000 * 8, 1024) == 251
