"""The MLP kernels' polynomial GELU, read from the kernel source, against
the exact GELU x Phi(x) (scipy's erfc) on the whole line, evaluated in the
kernel's FP32 order. Pins the constants: a dropped or mistyped coefficient,
a wrong clamp or a sign error breaks the 2.1e-4 bound."""
from __future__ import annotations

import os
import re

import numpy as np
from scipy.special import erfc

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_1805_06572_amd", "csrc", "fca_mlp.hip")


def kernel_gelu_constants():
    src = open(SRC).read()
    body = src[src.index("__device__ __forceinline__ float gelu(float x)"):]
    body = body[:body.index("\n}\n")]
    clamp = float(re.search(r"fminf\(fabsf\(x\), ([0-9.]+)f\)", body).group(1))
    first = float(re.search(r"float p = ([-0-9.e]+)f;", body).group(1))
    rest = [float(v) for v in re.findall(r"p = fmaf\(p, t, ([-0-9.e]+)f\);", body)]
    assert "return fmaf(-t, p, fmaxf(x, 0.0f));" in body
    return clamp, np.array(([first] + rest)[::-1], dtype=np.float32)  # low order first


def gelu_f32(x, T, c):
    x = np.asarray(x, dtype=np.float32)
    t = np.minimum(np.abs(x), np.float32(T))
    p = np.full_like(t, c[-1])
    for k in range(len(c) - 2, -1, -1):
        p = (p * t + c[k]).astype(np.float32)
    return (np.maximum(x, np.float32(0)) - t * p).astype(np.float64)


def test_kernel_gelu_within_bound_of_exact():
    T, c = kernel_gelu_constants()
    assert T == 4.0 and len(c) == 7
    x = np.linspace(-30.0, 30.0, 600001)
    exact = x * 0.5 * erfc(-x / np.sqrt(2.0))
    assert np.abs(gelu_f32(x, T, c) - exact).max() <= 2.1e-4


def test_kernel_gelu_special_values():
    T, c = kernel_gelu_constants()
    g = gelu_f32(np.array([0.0, 1e-3, -1e-3, 1.0, -1.0, 1e4, -1e4]), T, c)
    assert abs(g[0]) <= 1e-6                          # GELU(0) = 0
    assert abs(g[3] - 0.8413447460685429) <= 2.1e-4   # Phi(1)
    assert abs(g[4] + 0.15865525393145707) <= 2.1e-4  # -Phi(-1)
    assert abs(g[5] - 1e4) <= 1e-3 and abs(g[6]) <= 2.1e-4
