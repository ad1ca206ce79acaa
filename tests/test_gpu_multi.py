"""GPU parity of the J-source path (fca_multi_*: the approximate-joint-
diagonalisation EM for more than two sources) against the FP64 oracle
oracle/multi.py, through the C ABI. J = 2 is also checked against the
two-source C oracle and the two-source GPU path (the method reduces to
FastFCA there). Tolerances: per-frequency relative 1e-12 in FP64 (v, R,
log-likelihood, MMSE images; measured below 3e-15: the joint
diagonalisation's rotation order is the oracle's, its eigenvector arithmetic
is not); in FP32 bulk 1e-5 on v, R and the images and 1e-6 on the
log-likelihood after 4 iterations (measured below 2e-7 and 3e-8)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import multi
from paper_1805_06572_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def fca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_06572_amd import fca as mod
    mod.lib()
    return mod


def herm(A):
    return np.conj(np.swapaxes(A, -1, -2))


def per_freq_rel(a, b, axes):
    num = np.sqrt(np.sum(np.abs(a - b) ** 2, axis=axes))
    den = np.sqrt(np.sum(np.abs(b) ** 2, axis=axes))
    return num / np.maximum(den, 1e-300)


def j_source_mixture(J, M, F, N, seed):
    """y [F, N, M] = sum_j x_j with x_j(n, f) ~ CN(0, v_j R_j): R_j(f) = A A^H
    / tr + 0.05 I (A complex Gaussian), log v_j i.i.d. N(0, 1)."""
    rng = np.random.default_rng(seed)
    y = np.zeros((F, N, M), np.complex128)
    for j in range(J):
        for f in range(F):
            A = synth.cn(rng, (M, M))
            R = A @ herm(A)
            R = M * R / np.trace(R).real + 0.05 * np.eye(M)
            Lc = np.linalg.cholesky(R)
            v = np.exp(rng.standard_normal(N))
            y[f] += (np.sqrt(v)[:, None] * synth.cn(rng, (N, M))) @ Lc.T
    return y


def run_multi(fca, y, J, prec, iters, R0=None, v0=None):
    ctx = fca.fca_multi_init(torch.from_numpy(y).to(DEV), J, R0, v0, prec)
    try:
        ll, R, v = fca.fca_multi_em_step(ctx, iters)
        x = fca.fca_multi_separate(ctx)
        out = (ll.cpu().numpy(), R.cpu().numpy(), v.cpu().numpy().astype(np.float64),
               x.cpu().numpy().astype(np.complex128))
    finally:
        fca.fca_multi_destroy(ctx)
    return out


def check_against_oracle(fca, y, J, iters, prec, tol_v, tol_ll, R0=None, v0=None):
    S0d, v0d = multi.default_start(y, J)
    S0 = S0d if R0 is None else R0
    v0o = v0d if v0 is None else v0
    S, v, ll, P, lam = multi.fast_em(y, S0, v0o, iters)
    dt = np.float64 if prec == fca.FCA_FP64 else np.float32
    gll, gR, gv, gx = run_multi(fca, y.astype(np.complex128 if dt == np.float64 else np.complex64), J, prec, iters,
                                R0, None if v0 is None else v0.astype(dt))
    ev = per_freq_rel(gv, v, (-1,)).max()
    eR = per_freq_rel(gR, S, (-2, -1)).max()
    want_ll = ll[:iters].sum(1) if iters else ll[:1].sum(1)
    ell = np.max(np.abs(gll - want_ll) / np.abs(want_ll))
    x = multi.mmse(y, P, lam, v)
    ex = per_freq_rel(gx, x, (-2, -1)).max()
    print(f"J={J} M={y.shape[2]} N={y.shape[1]} prec={prec}: v {ev:.1e} R {eR:.1e} ll {ell:.1e} x {ex:.1e}")
    assert ev < tol_v and eR < tol_v and ex < tol_v
    assert ell < tol_ll
    return gll, gR, gv, gx


@pytest.mark.parametrize("J,M,F,N", [
    (3, 3, 4, 300),   # ragged: two frames per thread, 300 of 512 slots
    (4, 2, 3, 257),
    (3, 4, 3, 200),
    (4, 4, 2, 130),
    (3, 1, 3, 50),    # one microphone: the method is the exact EM
    (3, 2, 2, 1),     # a single frame
    (4, 3, 1, 2048),  # largest resident frame count (eight per thread)
])
def test_fp64_matches_oracle(fca, J, M, F, N):
    y = j_source_mixture(J, M, F, N, seed=100 * J + 10 * M + N)
    check_against_oracle(fca, y, J, 5, fca.FCA_FP64, 1e-12, 1e-12)


@pytest.mark.parametrize("J,M", [(3, 3), (4, 2), (4, 4)])
def test_fp32_bulk_matches_oracle(fca, J, M):
    y = j_source_mixture(J, M, 3, 400, seed=7 + J + M)
    check_against_oracle(fca, y, J, 4, fca.FCA_FP32_BULK, 1e-5, 1e-6)


def test_two_sources_equal_fastfca_and_the_c_oracle(fca):
    mx = synth.random_mixture(3, 4, 150, 11)
    S0, v0 = oracle.default_init(mx.y)
    S, v, ll, flags = oracle.em(mx.y, S0, v0, 6)
    assert not flags.any()
    gll, gR, gv, gx = run_multi(fca, mx.y, 2, fca.FCA_FP64, 6)
    assert per_freq_rel(gv, v, (-1,)).max() < 1e-10
    assert per_freq_rel(gR, S, (-2, -1)).max() < 1e-10
    np.testing.assert_allclose(gll, ll[:6].sum(1), rtol=1e-10)
    ctx = fca.fca_init(torch.from_numpy(mx.y).to(DEV), prec=fca.FCA_FP64)
    try:
        ll2, R2, v2 = fca.fca_em_step(ctx, 6)
        x2 = fca.fca_separate(ctx)[0].cpu().numpy()
    finally:
        fca.fca_destroy(ctx)
    assert per_freq_rel(gv, v2[0].cpu().numpy(), (-1,)).max() < 1e-10
    assert per_freq_rel(gx, x2, (-2, -1)).max() < 1e-10


def test_given_start_first_iteration_is_the_exact_em(fca):
    """From a jointly diagonalisable R0 the first iteration's E-step and power
    update are exact: v^(1) and the log-likelihood of theta^(0) equal those of
    the conventional J-source EM."""
    rng = np.random.default_rng(21)
    J, M, F, N = 3, 3, 3, 120
    y = j_source_mixture(J, M, F, N, seed=22)
    R0 = np.zeros((J, F, M, M), np.complex128)
    for f in range(F):
        Ai = np.linalg.inv(synth.cn(rng, (M, M)) + 2 * np.eye(M))
        for j in range(J):
            R0[j, f] = herm(Ai) @ np.diag(rng.uniform(0.3, 3.0, M)) @ Ai
    v0 = rng.uniform(0.2, 2.0, (J, F, N))
    _, ve, lle = multi.exact_em(y, R0, v0, 1)
    gll, _, gv, _ = run_multi(fca, y, J, fca.FCA_FP64, 1, R0, v0)
    assert per_freq_rel(gv, ve, (-1,)).max() < 1e-10
    np.testing.assert_allclose(gll[0], lle[0].sum(), rtol=1e-11)
    check_against_oracle(fca, y, J, 4, fca.FCA_FP64, 1e-12, 1e-12, R0=R0, v0=v0)


def test_images_sum_to_the_mixture_and_loglik_of_current_parameters(fca):
    J, M, F, N = 4, 3, 3, 90
    y = j_source_mixture(J, M, F, N, seed=5)
    ctx = fca.fca_multi_init(torch.from_numpy(y).to(DEV), J, prec=fca.FCA_FP64)
    try:
        ll, _, _ = fca.fca_multi_em_step(ctx, 3, want_R=False, want_v=False)
        ll0, _, _ = fca.fca_multi_em_step(ctx, 0, want_R=False, want_v=False)
        x = fca.fca_multi_separate(ctx).cpu().numpy()
    finally:
        fca.fca_multi_destroy(ctx)
    S0, v0 = multi.default_start(y, J)
    _, _, llo, _, _ = multi.fast_em(y, S0, v0, 3)
    np.testing.assert_allclose(ll.cpu().numpy(), llo[:3].sum(1), rtol=1e-10)
    np.testing.assert_allclose(ll0.cpu().numpy()[0], llo[3].sum(), rtol=1e-10)
    np.testing.assert_allclose(x.sum(0), y, rtol=0, atol=1e-12 * np.abs(y).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_calls_in_chunks_equal_one_call(fca, prec):
    """130 iterations in one call (two launches of at most 128) and as 100 +
    30 give bit-identical results: the state between launches is exactly the
    state the kernel keeps."""
    J, M, F, N = 3, 2, 3, 80
    p = fca.FCA_FP64 if prec == "fp64" else fca.FCA_FP32_BULK
    y = j_source_mixture(J, M, F, N, seed=9)
    yd = torch.from_numpy(y.astype(np.complex128 if prec == "fp64" else np.complex64)).to(DEV)
    res = []
    for split in ((130,), (100, 30)):
        ctx = fca.fca_multi_init(yd, J, prec=p)
        try:
            lls = []
            for it in split:
                ll, R, v = fca.fca_multi_em_step(ctx, it, allow_flags=True)
                lls.append(ll.cpu())
            res.append((torch.cat(lls).numpy(), R.cpu().numpy(), v.cpu().numpy()))
        finally:
            fca.fca_multi_destroy(ctx)
    for a, b in zip(res[0], res[1]):
        np.testing.assert_array_equal(a, b)


def test_argument_errors(fca):
    L = fca.lib()
    y = torch.zeros((2, 10, 2), dtype=torch.complex64, device=DEV)
    for J, shape in ((1, (2, 10, 2)), (5, (2, 10, 2)), (3, (2, 10, 5)), (3, (2, 2049, 2))):
        yy = torch.ones(shape, dtype=torch.complex64, device=DEV)
        with pytest.raises(fca.FcaError) as e:
            fca.fca_multi_init(yy, J)
        assert e.value.status == fca.FCA_E_ARG
    R0 = np.zeros((3, 2, 2, 2), np.complex128)
    R0[:] = np.eye(2)
    R0[2, 1] = np.diag([1.0, -1.0])   # R_J of frequency 1 not positive definite
    with pytest.raises(fca.FcaError) as e:
        fca.fca_multi_init(y, 3, R0=R0)
    assert e.value.status == fca.FCA_E_ARG and "positive definite" in str(e.value)
    R0[2, 1] = np.eye(2)
    R0[0, 1] = np.array([[1.0, 2.0], [2.0, 1.0]])   # R_1 of frequency 1 indefinite, positive diagonal
    with pytest.raises(fca.FcaError) as e:
        fca.fca_multi_init(y, 3, R0=R0)
    assert e.value.status == fca.FCA_E_ARG and "source 1 at frequency 1" in str(e.value)
    p, keep, _ = fca._problem(y, np.stack([np.eye(2)] * 2 * 2).reshape(2, 2, 2, 2).astype(np.complex128), None,
                              fca.FCA_FP32_BULK, None)
    import ctypes
    h = ctypes.c_void_p()
    assert L.fca_multi_init(ctypes.byref(p), 3, None, None, ctypes.byref(h)) == fca.FCA_E_ARG
    ctx = fca.fca_multi_init(y + 1, 3)
    try:
        assert L.fca_multi_em_step(ctx.handle, -1, None, None, None) == fca.FCA_E_ARG
        xh = np.zeros((3, 2, 10, 2), np.complex64)
        assert L.fca_multi_separate(ctx.handle, xh.ctypes.data) == fca.FCA_E_ARG
        assert "device" in L.fca_multi_last_error(ctx.handle).decode()
    finally:
        fca.fca_multi_destroy(ctx)
    del keep


def test_kernel_timing_counts_launches(fca):
    """fca_multi_timing: 130 iterations are two launches of the iteration
    kernel (at most 128 per launch), timed with events; the totals restart
    after each call and nothing is recorded while timing is off."""
    y = j_source_mixture(3, 2, 3, 64, seed=4)
    ctx = fca.fca_multi_init(torch.from_numpy(y.astype(np.complex64)).to(DEV), 3)
    try:
        assert fca.fca_multi_timing(ctx, True) == (0.0, 0)
        fca.fca_multi_em_step(ctx, 130, want_R=False, want_v=False, allow_flags=True)
        ms, n = fca.fca_multi_timing(ctx, False)
        assert n == 2 and ms > 0.0
        fca.fca_multi_em_step(ctx, 5, want_R=False, want_v=False, allow_flags=True)
        assert fca.fca_multi_timing(ctx, False) == (0.0, 0)
    finally:
        fca.fca_multi_destroy(ctx)
