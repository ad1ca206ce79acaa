"""Pins of the CPU oracle (conventional FCA EM, Section 2) to facts that do
not come from the oracle itself: a hand-worked example, textbook Gaussian
results, exact invariants of the EM, the paper's FastFCA equivalence claim,
and library density evaluations. CPU only."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import oracle
from paper_1805_06572_amd import synth
from tests.fastfca_numpy import fastfca

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def herm(A):
    return np.conj(np.swapaxes(A, -1, -2))


def random_problem(M, F, N, seed):
    mx = synth.random_mixture(M, F, N, seed)
    S0, v0 = oracle.default_init(mx.y)
    return mx, S0, v0


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ---------------------------------------------------------------- worked example
def test_hand_worked_single_mic_example():
    g = json.load(open(os.path.join(GOLDEN, "m1_two_frames.json")))
    y = np.array([complex(*c) for c in g["y"]]).reshape(1, 2, 1)
    S0 = np.array(g["S0"], dtype=np.complex128).reshape(2, 1, 1, 1)
    v0 = np.array(g["v0"]).reshape(2, 1, 2)
    S, v, ll, flags = oracle.em(y, S0, v0, 1)
    want_v = np.array([[a / b for a, b in row] for row in g["v1_num_den"]]).reshape(2, 1, 2)
    assert flags[0] == 0
    np.testing.assert_allclose(v, want_v, rtol=1e-15)
    np.testing.assert_allclose(S.real.ravel(), g["S1"], rtol=1e-15)
    ll0 = -2 * math.log(math.pi) - 2 * math.log(3) - 5 / 3
    ll1 = (-2 * math.log(math.pi) - math.log(17 / 9) - math.log(32 / 9) - 9 / 17 - 9 / 8)
    np.testing.assert_allclose(ll[:, 0], [ll0, ll1], rtol=1e-15)


# ---------------------------------------------------------------- textbook special case
def test_single_microphone_is_scalar_wiener_and_keeps_S():
    """M = 1: the E-step is the textbook scalar Gaussian posterior and the
    M-step leaves S_j unchanged at every iteration."""
    rng = np.random.default_rng(5)
    F, N = 3, 17
    y = synth.cn(rng, (F, N, 1))
    S0 = np.empty((2, F, 1, 1), np.complex128)
    S0[..., 0, 0] = rng.uniform(0.5, 2.0, (2, F))
    v0 = rng.uniform(0.1, 3.0, (2, F, N))
    S1, v1, _, _ = oracle.em(y, S0, v0, 1)
    s1 = v0[0] * S0[0, :, 0, 0, None].real
    s2 = v0[1] * S0[1, :, 0, 0, None].real
    post_var = s1 * s2 / (s1 + s2)
    m1 = s1 / (s1 + s2) * y[..., 0]
    m2 = s2 / (s1 + s2) * y[..., 0]
    want1 = (np.abs(m1) ** 2 + post_var) / S0[0, :, 0, 0, None].real
    want2 = (np.abs(m2) ** 2 + post_var) / S0[1, :, 0, 0, None].real
    np.testing.assert_allclose(v1[0], want1, rtol=1e-13)
    np.testing.assert_allclose(v1[1], want2, rtol=1e-13)
    S, _, _, _ = oracle.em(y, S0, v0, 15)
    np.testing.assert_allclose(S, S0, rtol=1e-12)


# ---------------------------------------------------------------- exact invariants
@pytest.mark.parametrize("M", [2, 3, 4])
def test_mstep_trace_identity(M):
    """tr(S_j^(l)^-1 S_j^(l+1)) = M exactly: v uses the old S, S the new v."""
    mx, S0, v0 = random_problem(M, 4, 40, 11)
    S, v = S0, v0
    for _ in range(4):
        Sn, vn, _, flags = oracle.em(mx.y, S, v, 1)
        assert not flags.any()
        tr = np.einsum("jfik,jfki->jf", np.linalg.inv(S), Sn)
        np.testing.assert_allclose(tr.real, M, rtol=1e-12)
        np.testing.assert_allclose(tr.imag, 0, atol=1e-12)
        S, v = Sn, vn


@pytest.mark.parametrize("M,seed", [(2, 0), (3, 1), (4, 2)])
def test_loglik_never_decreases(M, seed):
    mx, S0, v0 = random_problem(M, 6, 60, seed)
    _, _, ll, flags = oracle.em(mx.y, S0, v0, 25)
    assert not flags.any()
    tot = ll.sum(1)
    assert np.all(np.diff(tot) >= -1e-10 * np.abs(tot[1:]))
    assert tot[-1] > tot[0]


# ---------------------------------------------------------------- library density
def test_loglik_equals_library_gaussian_density():
    """The circular complex Gaussian CN(0, R) on C^M is the real Gaussian on
    R^2M with covariance [[Re R, -Im R], [Im R, Re R]] / 2."""
    mx, S0, v0 = random_problem(3, 2, 7, 3)
    S, v, ll, _ = oracle.em(mx.y, S0, v0, 2)
    for f in range(2):
        tot = 0.0
        for n in range(7):
            R = v[0, f, n] * S[0, f] + v[1, f, n] * S[1, f]
            cov = 0.5 * np.block([[R.real, -R.imag], [R.imag, R.real]])
            yv = mx.y[f, n]
            tot += multivariate_normal(mean=np.zeros(6), cov=cov).logpdf(np.r_[yv.real, yv.imag])
        np.testing.assert_allclose(ll[2, f], tot, rtol=1e-12)
    np.testing.assert_allclose(oracle.loglik(mx.y, S, v), ll[2], rtol=1e-14)


# ---------------------------------------------------------------- EM optimality
def test_one_iteration_maximises_expected_complete_loglik():
    """With the posterior taken from textbook Gaussian conditioning (Schur
    complement of the joint covariance of (x1, y)), the new v_j maximises the
    expected complete-data log-likelihood for the old S_j, and the new S_j
    maximises it for the new v_j: a perturbation either way lowers it."""
    M, F, N = 3, 2, 9
    mx, S0, v0 = random_problem(M, F, N, 7)
    Sn, vn, _, _ = oracle.em(mx.y, S0, v0, 1)
    rng = np.random.default_rng(0)
    for f in range(F):
        Phi = [[], []]
        for n in range(N):
            R1 = v0[0, f, n] * S0[0, f]
            R2 = v0[1, f, n] * S0[1, f]
            K = np.linalg.solve((R1 + R2).T, R1.T).T              # R1 (R1+R2)^-1
            mean1 = K @ mx.y[f, n]
            cov = R1 - K @ R1                                    # Schur complement
            cov = 0.5 * (cov + herm(cov))
            mean2 = mx.y[f, n] - mean1
            Phi[0].append(np.outer(mean1, np.conj(mean1)) + cov)
            Phi[1].append(np.outer(mean2, np.conj(mean2)) + cov)

        def q_term(vv, S, P):
            C = vv * S
            return -np.linalg.slogdet(C)[1] - np.trace(np.linalg.solve(C, P)).real

        for j in range(2):
            for n in range(N):
                q0 = q_term(vn[j, f, n], S0[j, f], Phi[j][n])
                for s in (1 - 1e-4, 1 + 1e-4):
                    assert q_term(vn[j, f, n] * s, S0[j, f], Phi[j][n]) < q0
            qS = sum(q_term(vn[j, f, n], Sn[j, f], Phi[j][n]) for n in range(N))
            for _ in range(4):
                H = synth.cn(rng, (M, M))
                H = 1e-4 * np.linalg.norm(Sn[j, f]) * (H + herm(H))
                for sgn in (-1, 1):
                    Sp = Sn[j, f] + sgn * H
                    assert sum(q_term(vn[j, f, n], Sp, Phi[j][n]) for n in range(N)) < qS


# ---------------------------------------------------------------- symmetries
def test_invertible_channel_transform_is_equivariant():
    """y -> A y with S0 -> A S0 A^H: same v, S -> A S A^H, and the
    log-likelihood shifts by -N log|det A|^2 per frequency."""
    M, F, N = 3, 3, 30
    mx, S0, v0 = random_problem(M, F, N, 9)
    A = synth.cn(np.random.default_rng(1), (F, M, M)) + 0.5 * np.eye(M)
    S, v, ll, _ = oracle.em(mx.y, S0, v0, 6)
    yA = np.einsum("fab,fnb->fna", A, mx.y)
    S0A = A[None] @ S0 @ herm(A)[None]
    SA, vA, llA, _ = oracle.em(yA, S0A, v0, 6)
    np.testing.assert_allclose(vA, v, rtol=1e-9)
    np.testing.assert_allclose(SA, A[None] @ S @ herm(A)[None], rtol=1e-9, atol=1e-9 * np.abs(SA).max())
    shift = -N * np.log(np.abs(np.linalg.det(A)) ** 2)
    np.testing.assert_allclose(llA, ll + shift[None, :], rtol=1e-10)


def test_source_swap_swaps_outputs():
    mx, S0, v0 = random_problem(3, 3, 25, 4)
    v0 = v0 * np.array([1.0, 1.7])[:, None, None]
    S, v, ll, _ = oracle.em(mx.y, S0, v0, 5)
    Ss, vs, lls, _ = oracle.em(mx.y, S0[::-1].copy(), v0[::-1].copy(), 5)
    np.testing.assert_allclose(Ss[::-1], S, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(vs[::-1], v, rtol=1e-11)
    np.testing.assert_allclose(lls, ll, rtol=1e-12)


def test_scale_exchange_between_S_and_v():
    mx, S0, v0 = random_problem(2, 3, 25, 6)
    S, v, ll, _ = oracle.em(mx.y, S0, v0, 5)
    Sc, vc, llc, _ = oracle.em(mx.y, 3.0 * S0, v0 / 3.0, 5)
    np.testing.assert_allclose(llc, ll, rtol=1e-12)
    np.testing.assert_allclose(vc[..., None, None] * Sc[:, :, None], v[..., None, None] * S[:, :, None],
                               rtol=1e-10, atol=1e-12)


def test_frequency_subset_is_an_exact_subproblem():
    mx, S0, v0 = random_problem(2, 8, 20, 8)
    S, v, ll, _ = oracle.em(mx.y, S0, v0, 4)
    idx = [1, 5, 6]
    Ss, vs, lls, _ = oracle.em(mx.y[idx], S0[:, idx], v0[:, idx], 4)
    np.testing.assert_array_equal(Ss, S[:, idx])
    np.testing.assert_array_equal(vs, v[:, idx])
    np.testing.assert_array_equal(lls, ll[:, idx])


# ---------------------------------------------------------------- paper's equivalence claim
def test_conventional_equals_fastfca_on_random_workload():
    """The paper's strict-equivalence claim, checked against an independent
    numpy/LAPACK FastFCA on the small random workload (M=2, F=257, N=200,
    20 iterations from the plain start)."""
    mx = synth.random_mixture(2, 257, 200, 0)
    S0, v0 = oracle.default_init(mx.y)
    S, v, ll, flags = oracle.em(mx.y, S0, v0, 20)
    Sf, vf, llf = fastfca(mx.y, S0, v0, 20)
    assert not flags.any()
    for j in range(2):
        err_v = np.linalg.norm(v[j] - vf[j], axis=-1) / np.linalg.norm(vf[j], axis=-1)
        assert err_v.max() < 1e-10
        err_S = np.linalg.norm(S[j] - Sf[j], axis=(-2, -1)) / np.linalg.norm(Sf[j], axis=(-2, -1))
        assert err_S.max() < 1e-10
    np.testing.assert_allclose(ll.sum(1), llf.sum(1), rtol=1e-12)


@pytest.mark.parametrize("M", [3, 4])
def test_conventional_equals_fastfca_larger_arrays(M):
    mx = synth.random_mixture(M, 12, 80, 20 + M)
    S0, v0 = oracle.default_init(mx.y)
    S, v, ll, _ = oracle.em(mx.y, S0, v0, 10)
    Sf, vf, llf = fastfca(mx.y, S0, v0, 10)
    np.testing.assert_allclose(v, vf, rtol=1e-9)
    np.testing.assert_allclose(S, Sf, rtol=1e-9, atol=1e-10 * np.abs(Sf).max())
    np.testing.assert_allclose(ll, llf, rtol=1e-11)


# ---------------------------------------------------------------- MMSE output
def test_mmse_images_sum_to_mixture_and_match_wiener():
    mx, S0, v0 = random_problem(3, 3, 12, 2)
    S, v, _, _ = oracle.em(mx.y, S0, v0, 3)
    x = oracle.mmse(mx.y, S, v)
    np.testing.assert_allclose(x[0] + x[1], mx.y, rtol=1e-12, atol=1e-12)
    # textbook multichannel Wiener filter for a single bin
    f, n = 1, 4
    R1 = v[0, f, n] * S[0, f]
    R2 = v[1, f, n] * S[1, f]
    np.testing.assert_allclose(x[0, f, n], R1 @ np.linalg.solve(R1 + R2, mx.y[f, n]), rtol=1e-12)


# ---------------------------------------------------------------- failure handling
def test_non_pd_start_is_flagged_and_frozen():
    mx, S0, v0 = random_problem(2, 4, 10, 1)
    S0 = S0.copy()
    S0[1, 2] = np.diag([1.0, -1.0])                 # not positive definite at f = 2
    S, v, ll, flags = oracle.em(mx.y, S0, v0, 3)
    assert flags[2] == oracle.FLAG_NOT_PD
    assert not flags[[0, 1, 3]].any()
    assert np.all(np.isnan(ll[:, 2])) and np.all(np.isfinite(ll[:, [0, 1, 3]]))
    Sr, vr, llr, _ = oracle.em(mx.y[[0, 1, 3]], S0[:, [0, 1, 3]], v0[:, [0, 1, 3]], 3)
    np.testing.assert_array_equal(vr, v[:, [0, 1, 3]])
    np.testing.assert_array_equal(v[:, 2], v0[:, 2])   # frozen at the start
