"""fca_em_solve_noalloc (the plain-start EM of one mixture with no device
allocation, its state in the library's fixed device array) against the
context path it is a variant of, fca_init + fca_em_step, through the C ABI:
two calls in a row, the second on a smaller input, then a caller-given start;
FP64 within relative 1e-10, FP32 bulk within relative 1e-4."""
from __future__ import annotations

import numpy as np
import pytest

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


def per_freq_rel(a, b, axes):
    return np.sqrt(np.sum(np.abs(a - b) ** 2, axis=axes)) / np.sqrt(np.sum(np.abs(b) ** 2, axis=axes))


def context_run(fca, y, prec, iters, v0=None):
    ctx = fca.fca_init(torch.from_numpy(y).to(DEV), v0=v0, prec=prec)
    try:
        ll, R, v = fca.fca_em_step(ctx, iters, allow_flags=True)
        flags = fca.fca_status_per_freq(ctx)[0]
    finally:
        fca.fca_destroy(ctx)
    return ll.cpu().numpy()[0], R[0].cpu().numpy(), v[0].cpu().numpy(), flags


def noalloc_run(fca, y, prec, iters, pitch, v0=None):
    F, N, M = y.shape
    cdt = np.complex128 if prec == fca.FCA_FP64 else np.complex64
    rdt = torch.float64 if prec == fca.FCA_FP64 else torch.float32
    yl = np.zeros((F, M, pitch), cdt)
    yl[:, :, :N] = np.transpose(y, (0, 2, 1))
    yl[:, :, N:] = 7.0                                    # padding is never read
    yd = torch.from_numpy(yl).to(DEV)
    v = torch.full((2, F, pitch), -1.0, dtype=rdt, device=DEV)
    if v0 is not None:
        v[:, :, :N] = torch.from_numpy(np.asarray(v0)).to(device=DEV, dtype=rdt)
    ll = torch.empty(max(iters, 1), dtype=torch.float64, device=DEV)
    R = torch.empty((2, F, M, M), dtype=torch.complex128, device=DEV)
    flags = torch.full((F,), -1, dtype=torch.int32, device=DEV)
    fca.fca_em_solve_noalloc(yd, v, N, iters, use_v0=v0 is not None, loglik=ll, R_out=R, flags_out=flags)
    torch.cuda.synchronize()
    return ll.cpu().numpy(), R.cpu().numpy(), v[:, :, :N].cpu().numpy(), flags.cpu().numpy()


def check(got, want, tol):
    gll, gR, gv, gf = got
    ll, R, v, f = want
    np.testing.assert_array_equal(gf, f)
    np.testing.assert_allclose(gll, ll, rtol=tol)
    assert per_freq_rel(gv.astype(np.float64), v.astype(np.float64), (-1,)).max() < tol
    assert per_freq_rel(gR, R, (-2, -1)).max() < tol


def test_noalloc_equals_context_path_twice(fca):
    big = synth.array_mixture(4, 65, 700, seed=61, complex64=True).y
    small = synth.random_mixture(3, 9, 130, seed=62).y
    got = noalloc_run(fca, big, fca.FCA_FP32_BULK, 9, pitch=704)
    check(got, context_run(fca, big, fca.FCA_FP32_BULK, 9), 1e-4)
    got = noalloc_run(fca, small, fca.FCA_FP64, 5, pitch=130)
    check(got, context_run(fca, small, fca.FCA_FP64, 5), 1e-10)


def test_noalloc_given_start_and_eval_only(fca):
    mx = synth.random_mixture(2, 17, 257, seed=63)
    v0 = 0.5 * mx.v + 0.01
    check(noalloc_run(fca, mx.y, fca.FCA_FP64, 4, pitch=320, v0=v0),
          context_run(fca, mx.y, fca.FCA_FP64, 4, v0=v0), 1e-10)
    check(noalloc_run(fca, mx.y, fca.FCA_FP64, 0, pitch=257),
          context_run(fca, mx.y, fca.FCA_FP64, 0), 1e-10)


def test_noalloc_argument_errors(fca):
    L = fca.lib()
    y = torch.zeros((4, 2, 64), dtype=torch.complex64, device=DEV)
    v = torch.ones((2, 4, 64), dtype=torch.float32, device=DEV)
    yh = np.zeros((4, 2, 64), np.complex64)
    cases = [(2, 2049, 64, 64), (2, 4, 2049, 4096), (9, 4, 64, 64), (2, 4, 65, 64)]
    for M, F, N, pitch in cases:
        st = L.fca_em_solve_noalloc(M, F, N, fca.FCA_FP32_BULK, y.data_ptr(), pitch, v.data_ptr(), 0, 3,
                                    None, None, None, None)
        assert st == fca.FCA_E_ARG, (M, F, N, pitch)
    st = L.fca_em_solve_noalloc(2, 4, 64, fca.FCA_FP32_BULK, yh.ctypes.data, 64, v.data_ptr(), 0, 3,
                                None, None, None, None)
    assert st == fca.FCA_E_ARG and "device" in fca.fca_last_error()
