"""More pins of the CPU oracle against values it does not produce itself:
hand-worked fixtures for the plain start, the MMSE images and the learned-
start network's forward pass, and a 50-digit brute-force EM (mpmath) on tiny
inputs that takes the posterior from textbook Gaussian conditioning rather
than from the oracle's formulas. CPU only."""
from __future__ import annotations

import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1805_06572_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return json.load(open(os.path.join(GOLDEN, name)))


# ---------------------------------------------------------------- plain start
def test_default_init_hand_worked():
    """Algorithm 1, step 1 with the plain start: exact powers (silent bins
    at the floor of 1e-12 times the mean power) and the two covariances."""
    g = _load("default_init_two_mics.json")
    M, F, N = g["M"], g["F"], g["N"]
    y = np.array([[[complex(*c) for c in frame] for frame in row] for row in g["y"]])
    assert y.shape == (F, N, M)
    S0, v0 = oracle.default_init(y)
    floor = g["floor_scale"] * g["floor_num_den"][0] / g["floor_num_den"][1]
    want = np.array([[floor if nd is None else nd[0] / nd[1] for nd in row] for row in g["v_num_den"]])
    for j in range(2):
        np.testing.assert_allclose(v0[j], want, rtol=1e-15)
    R2 = np.array([[nd[0] / nd[1] for nd in row] for row in g["R2_num_den"]])
    for f in range(F):
        np.testing.assert_array_equal(S0[0, f], np.array(g["R1"], dtype=np.complex128))
        np.testing.assert_array_equal(S0[1, f], R2.astype(np.complex128))


def test_default_init_silent_mixture_uses_unit_floor():
    """All bins silent: the mean power is 0 and every power becomes 1."""
    S0, v0 = oracle.default_init(np.zeros((3, 5, 2), np.complex128))
    np.testing.assert_array_equal(v0, np.ones((2, 3, 5)))
    np.testing.assert_array_equal(S0[1, 0], np.array([[1.5, 0], [0, 1]], np.complex128))


# ---------------------------------------------------------------- MMSE on the M = 1 example
def test_mmse_hand_worked_single_mic_example():
    """eq. (MMSE) on the hand-worked single-microphone example: with
    S1 = 1, S2 = 2 and v1 = v2 = 1 the mixture variance is 3, so
    mu1 = y/3 and mu2 = 2y/3."""
    g = _load("m1_two_frames.json")
    y = np.array([complex(*c) for c in g["y"]]).reshape(1, 2, 1)
    S0 = np.array(g["S0"], dtype=np.complex128).reshape(2, 1, 1, 1)
    v0 = np.array(g["v0"]).reshape(2, 1, 2)
    x = oracle.mmse(y, S0, v0)
    np.testing.assert_allclose(x[0, 0, :, 0], y[0, :, 0] / 3, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(x[1, 0, :, 0], 2 * y[0, :, 0] / 3, rtol=1e-15, atol=1e-16)


# ---------------------------------------------------------------- network forward pass
def _tiny_params(g):
    H = g["H"]
    W1 = np.zeros((H, mlp.KP))
    for r, c, val in g["layer1_nonzero"]:
        W1[r, c] = val
    parts = [W1.ravel(), g["b1"], np.ravel(g["W2"]), g["b2"], np.ravel(g["W3"]), g["b3"], g["w4"],
             [math.log(3.0) - 1.0]]
    p = np.concatenate([np.asarray(a, dtype=np.float64) for a in parts])
    assert p.size == mlp.num_params(H)
    return p


def test_mlp_forward_hand_worked():
    """Three GELU layers and the sigmoid output on chosen weights: the
    pre-activations and r worked out by hand (GELU(a) - GELU(-a) = a, and a
    normal-table value for bin B)."""
    g = _load("mlp_forward_tiny.json")
    p = _tiny_params(g)
    ys = np.array([[complex(*c) for c in b["y"]] for b in g["bins"]])
    fpos = np.array([b["fpos"] for b in g["bins"]])
    X = mlp.features(ys, fpos)
    r, (pres, _, z) = mlp.forward(p, X)
    for k, b in enumerate(g["bins"]):
        for layer in range(3):
            np.testing.assert_allclose(pres[layer][k], b["pre"][layer], rtol=0, atol=1e-15)
    np.testing.assert_allclose(z[0], math.log(3.0), rtol=1e-15)
    np.testing.assert_allclose(r[0], g["bins"][0]["r"], rtol=1e-15)
    zb = g["bins"][1]["z_minus_ln3_plus_1"] + math.log(3.0) - 1.0
    np.testing.assert_allclose(z[1], zb, rtol=1e-15)
    np.testing.assert_allclose(r[1], 1.0 / (1.0 + math.exp(-zb)), rtol=1e-15)


# ---------------------------------------------------------------- 50-digit brute force
def _mp_em(y, S0, v0, iters):
    """Conventional EM on tiny inputs in 50-digit arithmetic. The posterior
    of x1 given y = x1 + x2 is textbook conditioning of jointly Gaussian
    vectors: mean K y and covariance C1 - K C1 with C_j = v_j S_j and
    K = C1 (C1 + C2)^-1; x2 has mean y - K y and the same covariance. The
    M-step maximises the expected complete-data log-likelihood: v_j for the
    old S_j (tr(S_j^-1 Phi_j)/M), then S_j for the new v_j (mean of
    Phi_j / v_j). The log-likelihood of theta is log CN(y; 0, C1 + C2) with
    the determinant and inverse taken by mpmath's elimination."""
    F, N, M = y.shape
    S = [[mp.matrix([[mp.mpc(complex(S0[j, f, a, b])) for b in range(M)] for a in range(M)])
          for f in range(F)] for j in range(2)]
    v = [[[mp.mpf(float(v0[j, f, n])) for n in range(N)] for f in range(F)] for j in range(2)]
    lls = []
    for it in range(iters + 1):
        ll = [mp.mpf(0)] * F
        newS = [[None] * F for _ in range(2)]
        newv = [[[None] * N for _ in range(F)] for _ in range(2)]
        for f in range(F):
            Sinv = [mp.inverse(S[j][f]) for j in range(2)]
            Phis = [[], []]
            for n in range(N):
                yv = mp.matrix([mp.mpc(complex(y[f, n, m])) for m in range(M)])
                C1 = S[0][f] * v[0][f][n]
                C2 = S[1][f] * v[1][f][n]
                R = C1 + C2
                Ri = mp.inverse(R)
                quad = (yv.H * Ri * yv)[0].real
                ll[f] += -M * mp.log(mp.pi) - mp.log(mp.re(mp.det(R))) - quad
                K = C1 * Ri
                mu1 = K * yv
                mu2 = yv - mu1
                cov = C1 - K * C1
                for j, mu in ((0, mu1), (1, mu2)):
                    Phi = mu * mu.H + cov
                    Phis[j].append(Phi)
                    tr = sum((Sinv[j] * Phi)[i, i] for i in range(M))
                    newv[j][f][n] = mp.re(tr) / M
            for j in range(2):
                acc = mp.zeros(M, M)
                for n in range(N):
                    acc += Phis[j][n] / newv[j][f][n]
                newS[j][f] = acc / N
        lls.append(ll)
        if it < iters:
            S, v = newS, newv
    return S, v, lls


@pytest.mark.parametrize("M,N,iters,seed", [(2, 4, 3, 0), (3, 3, 3, 1), (2, 1, 2, 2), (3, 4, 2, 3)])
def test_oracle_matches_50_digit_brute_force(M, N, iters, seed):
    """The oracle (FP64, Cholesky solves, the paper's posterior formula)
    against the 50-digit brute force above on random tiny inputs from a
    random start: every iterate's powers, covariances and log-likelihood."""
    mp.mp.dps = 50
    rng = np.random.default_rng(100 + seed)
    F = 2
    y = synth.cn(rng, (F, N, M))
    S0 = np.empty((2, F, M, M), np.complex128)
    for j in range(2):
        for f in range(F):
            A = synth.cn(rng, (M, M))
            S0[j, f] = A @ A.conj().T + 0.5 * np.eye(M)
    v0 = rng.uniform(0.3, 2.0, (2, F, N))
    S, v, ll, flags = oracle.em(y, S0, v0, iters)
    assert not flags.any()
    Smp, vmp, llmp = _mp_em(y, S0, v0, iters)
    want_v = np.array([[[float(vmp[j][f][n]) for n in range(N)] for f in range(F)] for j in range(2)])
    want_S = np.array([[[[complex(Smp[j][f][a, b]) for b in range(M)] for a in range(M)] for f in range(F)]
                       for j in range(2)])
    want_ll = np.array([[float(l) for l in row] for row in llmp])
    np.testing.assert_allclose(v, want_v, rtol=1e-12)
    np.testing.assert_allclose(S, want_S, rtol=1e-12, atol=1e-13 * np.abs(want_S).max())
    np.testing.assert_allclose(ll, want_ll, rtol=1e-12)
