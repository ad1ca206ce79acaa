"""FP64 reference of the learned-initialisation network -- TEST INFRASTRUCTURE.

Only tests may import this module. It restates, in plain numpy, the network
that the library's MLP kernels compute (the library's header documents it):
features of a bin y in C^M, three hidden layers of width H with the erf
form of GELU, a sigmoid output r, and the mean binary cross-entropy against
soft targets, with its gradient by reverse-mode differentiation. Parameters
use the library's flat layout (per hidden layer: weight [H][in] then bias
[H], in = 32 padded inputs for the first layer; then output weight [H] and
bias [1]); H follows from the length, 2 H^2 + 36 H + 1.

``bf16=True`` evaluates the same network with the storage the library's
kernels use: the hidden-layer weight matrices, the features and the first
two layers' GELU outputs are rounded to BF16 (round to nearest even) before
they enter a product; biases, the output weights, every pre-activation and
the third layer's GELU output stay unrounded. In the backward pass the
per-layer deltas (loss gradient with respect to the pre-activations) are
rounded to BF16 as well. Everything else is FP64.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

KP = 32


def num_params(hidden: int) -> int:
    return KP * hidden + hidden + 2 * (hidden * hidden + hidden) + hidden + 1


def hidden_width(n_params: int) -> int:
    """H with num_params(H) == n_params."""
    h = int(round((-(KP + 4) + np.sqrt((KP + 4) ** 2 - 8 * (1 - n_params))) / 4))
    if num_params(h) != n_params:
        raise ValueError(f"{n_params} parameters fit no hidden width")
    return h


def unpack(params: np.ndarray):
    p = np.asarray(params, dtype=np.float64)
    H = hidden_width(p.size)
    Ws, bs, o = [], [], 0
    for l in range(3):
        fan = KP if l == 0 else H
        Ws.append(p[o:o + H * fan].reshape(H, fan))
        o += H * fan
        bs.append(p[o:o + H])
        o += H
    w4 = p[o:o + H]
    o += H
    b4 = p[o]
    return Ws, bs, w4, b4


def features(y: np.ndarray, fpos: np.ndarray) -> np.ndarray:
    """[n, 32]: log(|y_m|^2 + 1e-20); cos, sin of angle(y_m) - angle(y_1); f/(F-1); zeros."""
    y = np.asarray(y, dtype=np.complex128)
    n, M = y.shape
    X = np.zeros((n, KP))
    X[:, :M] = np.log(np.abs(y) ** 2 + 1e-20)
    rel = y[:, 1:] * np.conj(y[:, :1])
    mag = np.abs(rel)
    ok = mag > 0
    X[:, M:M + 2 * (M - 1):2] = np.where(ok, rel.real / np.where(ok, mag, 1), 0)
    X[:, M + 1:M + 2 * (M - 1):2] = np.where(ok, rel.imag / np.where(ok, mag, 1), 0)
    X[:, 3 * M - 2] = fpos
    return X


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def _q(a, on):
    return bf16_round(a).astype(np.float64) if on else a


def forward(params, X, bf16=False):
    """(r [n], cache) for features X [n, 32]."""
    Ws, bs, w4, b4 = unpack(params)
    if bf16:
        Ws = [_q(W, True) for W in Ws]
    h = _q(X, bf16)
    pres, hs = [], [h]
    for l, (W, b) in enumerate(zip(Ws, bs)):
        a = h @ W.T + b
        pres.append(a)
        h = _q(gelu(a), bf16 and l < 2)
        hs.append(h)
    z = h @ w4 + b4
    r = 1.0 / (1.0 + np.exp(-z))
    return r, (pres, hs, z)


def loss(params, X, t, bf16=False):
    r, (_, _, z) = forward(params, X, bf16)
    sp_neg = np.logaddexp(0.0, -z)   # -log r
    sp_pos = np.logaddexp(0.0, z)    # -log(1 - r)
    return float(np.mean(t * sp_neg + (1.0 - t) * sp_pos))


def loss_and_grad(params, X, t, bf16=False):
    """Mean binary cross-entropy and its gradient (flat, same layout)."""
    Ws, bs, w4, b4 = unpack(params)
    if bf16:
        Ws = [_q(W, True) for W in Ws]
    r, (pres, hs, z) = forward(params, X, bf16)
    n = X.shape[0]
    dz = (r - t) / n
    g_w4 = hs[-1].T @ dz
    g_b4 = dz.sum()
    d = _q(np.outer(dz, w4) * gelu_grad(pres[-1]), bf16)
    gW, gb = [None] * 3, [None] * 3
    for l in (2, 1, 0):
        gW[l] = d.T @ hs[l]
        gb[l] = d.sum(0)
        if l > 0:
            d = _q((d @ Ws[l]) * gelu_grad(pres[l - 1]), bf16)
    parts = []
    for l in range(3):
        parts += [gW[l].ravel(), gb[l]]
    parts += [g_w4, np.array([g_b4])]
    return loss(params, X, t, bf16), np.concatenate(parts)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest even) and back."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)
