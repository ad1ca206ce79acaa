"""Pins of the J-source oracles (oracle/multi.py): the approximate-joint-
diagonalisation EM against the two-source C oracle (the paper's
equivalence), against the exact J-source EM where it is exact (one
microphone; the first iteration from a jointly diagonalisable start), its
AJD against LAPACK and jointly diagonalisable inputs; the exact J-source EM
against the C oracle, a 50-digit brute force with the information-form
posterior, and monotone likelihood. CPU only."""
from __future__ import annotations

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import multi
from paper_1805_06572_amd import synth


def herm(A):
    return np.conj(np.swapaxes(A, -1, -2))


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def jd_start(rng, J, F, M):
    """S_j = A^-H Lambda_j A^-1 with one A per frequency: jointly
    diagonalisable."""
    S = np.zeros((J, F, M, M), np.complex128)
    for f in range(F):
        A = synth.cn(rng, (M, M)) + 2 * np.eye(M)
        Ai = np.linalg.inv(A)
        for j in range(J):
            S[j, f] = herm(Ai) @ np.diag(rng.uniform(0.3, 3.0, M)) @ Ai
    return S


def test_two_sources_equal_the_c_oracle():
    mx = synth.random_mixture(2, 5, 60, 3)
    S0, v0 = oracle.default_init(mx.y)
    S0m, v0m = multi.default_start(mx.y, 2)
    np.testing.assert_array_equal(S0m, S0)
    np.testing.assert_allclose(v0m, v0, rtol=1e-15)
    S, v, ll, flags = oracle.em(mx.y, S0, v0, 8)
    Sm, vm, llm, _, _ = multi.fast_em(mx.y, S0, v0, 8)
    assert not flags.any()
    assert rel(vm, v) < 1e-10 and rel(Sm, S) < 1e-10
    np.testing.assert_allclose(llm, ll, rtol=1e-11)
    Se, ve, lle = multi.exact_em(mx.y, S0, v0, 8)
    assert rel(ve, v) < 1e-10 and rel(Se, S) < 1e-10
    np.testing.assert_allclose(lle, ll, rtol=1e-11)


def test_one_microphone_equals_the_exact_em():
    rng = np.random.default_rng(4)
    J, F, N = 3, 3, 20
    y = synth.cn(rng, (F, N, 1))
    S0 = rng.uniform(0.5, 2.0, (J, F, 1, 1)).astype(np.complex128)
    v0 = rng.uniform(0.2, 2.0, (J, F, N))
    S, v, ll = multi.exact_em(y, S0, v0, 6)
    Sf, vf, llf, _, _ = multi.fast_em(y, S0, v0, 6)
    np.testing.assert_allclose(vf, v, rtol=1e-12)
    np.testing.assert_allclose(Sf, S, rtol=1e-12)
    np.testing.assert_allclose(llf, ll, rtol=1e-12)


@pytest.mark.parametrize("J,M", [(3, 3), (4, 2)])
def test_first_iteration_from_a_jointly_diagonalisable_start_is_exact(J, M):
    rng = np.random.default_rng(10 + J)
    F, N = 2, 30
    y = synth.cn(rng, (F, N, M))
    S0 = jd_start(rng, J, F, M)
    v0 = rng.uniform(0.2, 2.0, (J, F, N))
    _, v, ll = multi.exact_em(y, S0, v0, 1)
    _, vf, llf, _, _ = multi.fast_em(y, S0, v0, 1)
    np.testing.assert_allclose(vf, v, rtol=1e-11)
    np.testing.assert_allclose(llf[0], ll[0], rtol=1e-12)


def test_ajd_of_one_matrix_is_its_eigendecomposition():
    rng = np.random.default_rng(5)
    for M in (2, 3, 4, 5):
        A = synth.cn(rng, (M, M))
        A = A @ herm(A)
        U, Cs, _ = multi.ajd([A], 1e-15)
        np.testing.assert_allclose(herm(U) @ U, np.eye(M), atol=1e-14)
        np.testing.assert_allclose(np.abs(Cs[0] - np.diag(np.diag(Cs[0]))).max(), 0, atol=1e-13)
        w = np.linalg.eigvalsh(A)
        np.testing.assert_allclose(np.sort(np.diag(Cs[0]).real), w, rtol=0, atol=1e-13 * w.max())


def test_ajd_diagonalises_jointly_diagonalisable_matrices_and_reduces_the_criterion():
    rng = np.random.default_rng(6)
    M = 4
    Q, _ = np.linalg.qr(synth.cn(rng, (M, M)))
    Ms = [Q @ np.diag(rng.uniform(0.5, 3, M)) @ herm(Q) for _ in range(3)]
    _, Cs, _ = multi.ajd(Ms, 1e-15)
    assert max(np.abs(C - np.diag(np.diag(C))).max() for C in Cs) < 1e-13

    def off(Cs):
        return sum(np.sum(np.abs(C - np.diag(np.diag(C))) ** 2) for C in Cs)
    Ms = []
    for _ in range(3):
        A = synth.cn(rng, (M, M))
        Ms.append(A @ herm(A))
    before = off(Ms)
    for p, q in ((0, 1), (2, 3), (0, 2), (1, 3), (0, 3), (1, 2)):
        c, s = multi.cs_rotation(Ms, p, q)
        Ms2 = [multi.rotate(C, p, q, c, s)[0] for C in Ms]
        assert off(Ms2) <= off(Ms) + 1e-12
        Ms = Ms2
    assert off(Ms) < before


def _mp_em(y, S0, v0, iters):
    """Exact J-source EM in 50 digits with the posterior covariance in
    information form, (R_j^-1 + (sum_{k != j} R_k)^-1)^-1, and the mean
    R_j (sum_k R_k)^-1 y."""
    F, N, M = y.shape
    J = S0.shape[0]
    S = [[mp.matrix([[mp.mpc(complex(S0[j, f, a, b])) for b in range(M)] for a in range(M)]) for f in range(F)]
         for j in range(J)]
    v = [[[mp.mpf(float(v0[j, f, n])) for n in range(N)] for f in range(F)] for j in range(J)]
    lls = []
    for it in range(iters + 1):
        ll = [mp.mpf(0)] * F
        nS = [[None] * F for _ in range(J)]
        nv = [[[None] * N for _ in range(F)] for _ in range(J)]
        for f in range(F):
            Si = [mp.inverse(S[j][f]) for j in range(J)]
            Phis = [[] for _ in range(J)]
            for n in range(N):
                yv = mp.matrix([mp.mpc(complex(y[f, n, m])) for m in range(M)])
                Rs = [S[j][f] * v[j][f][n] for j in range(J)]
                R = Rs[0]
                for k in range(1, J):
                    R = R + Rs[k]
                Ri = mp.inverse(R)
                ll[f] += -M * mp.log(mp.pi) - mp.log(mp.re(mp.det(R))) - (yv.H * Ri * yv)[0].real
                for j in range(J):
                    other = None
                    for k in range(J):
                        if k != j:
                            other = Rs[k] if other is None else other + Rs[k]
                    cov = mp.inverse(mp.inverse(Rs[j]) + mp.inverse(other))
                    mu = Rs[j] * Ri * yv
                    Phi = mu * mu.H + cov
                    Phis[j].append(Phi)
                    nv[j][f][n] = mp.re(sum((Si[j] * Phi)[i, i] for i in range(M))) / M
            for j in range(J):
                acc = mp.zeros(M, M)
                for n in range(N):
                    acc += Phis[j][n] / nv[j][f][n]
                nS[j][f] = acc / N
        lls.append(ll)
        if it < iters:
            S, v = nS, nv
    return S, v, lls


def test_exact_em_matches_50_digit_brute_force():
    mp.mp.dps = 50
    rng = np.random.default_rng(7)
    J, F, N, M = 3, 1, 3, 2
    y = synth.cn(rng, (F, N, M))
    S0 = jd_start(rng, J, F, M) + 0.2 * np.eye(M)
    v0 = rng.uniform(0.3, 2.0, (J, F, N))
    S, v, ll = multi.exact_em(y, S0, v0, 2)
    Smp, vmp, llmp = _mp_em(y, S0, v0, 2)
    np.testing.assert_allclose(v, [[[float(vmp[j][f][n]) for n in range(N)] for f in range(F)] for j in range(J)],
                               rtol=1e-12)
    np.testing.assert_allclose(S, [[[[complex(Smp[j][f][a, b]) for b in range(M)] for a in range(M)]
                                    for f in range(F)] for j in range(J)], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ll, [[float(x) for x in row] for row in llmp], rtol=1e-12)


def test_exact_em_likelihood_never_decreases():
    rng = np.random.default_rng(8)
    J, F, N, M = 3, 2, 40, 3
    y = synth.cn(rng, (F, N, M))
    S0, v0 = multi.default_start(y, J)
    _, _, ll = multi.exact_em(y, S0, v0, 10)
    tot = ll.sum(1)
    assert np.all(np.diff(tot) >= -1e-10 * np.abs(tot[1:]))
