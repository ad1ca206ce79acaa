"""GPU parity of fca_set_mask_covariances (mask-weighted initial covariances, one
wave per mixture and frequency) against the oracle's plain definition
(oracle/mask_init.py), through the C ABI. The start is read back as the R of
theta^(0) recovered from its generalized eigendecomposition, so the
tolerance (relative 1e-9) covers that round trip in FP64."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import mask_init

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


def _mixtures(F, shapes, seed, silent_f=None):
    rng = np.random.default_rng(seed)
    ys, v0s = [], []
    for M, N in shapes:
        y = (rng.standard_normal((F, N, M)) + 1j * rng.standard_normal((F, N, M))).astype(np.complex64)
        if silent_f is not None:
            y[silent_f] = 0
        ys.append(y)
        v0s.append(rng.gamma(0.5, 1.0, size=(2, F, N)).astype(np.float32) + np.float32(1e-3))
    return ys, v0s


def _start_R(fca, ctx):
    _, R, _ = fca.fca_em_step(ctx, 0, want_loglik=False, want_v=False, allow_flags=True)
    return [r.cpu().numpy() for r in R]


def _default_R(M, F):
    R = np.zeros((2, F, M, M), dtype=np.complex128)
    R[:] = np.eye(M)
    R[1, :, 0, 0] += 0.5
    return R


@pytest.mark.parametrize("prec,shapes,p", [
    ("fp32", [(4, 300), (2, 1), (8, 257), (4, 1000), (1, 50)], 3.0),
    ("fp64", [(1, 40), (4, 300), (2, 1), (8, 257), (4, 1000)], 3.0),
    ("fp32", [(4, 300), (4, 77), (4, 1), (2, 40), (2, 513), (8, 90)], 2.5),
    ("fp64", [(3, 64), (3, 65), (5, 200), (6, 31), (7, 10)], 1.0)])
def test_mask_start_matches_oracle(fca, prec, shapes, p):
    """Mixtures of M = 1..8 with uneven N (ragged against the 64-frame
    workgroup, single-frame mixtures), runs of equal M (one decomposition
    launch each) and a silent frequency; integer, fractional and no
    sharpening; the masks come from seeded powers given as v0."""
    F, load = 9, 1e-3
    ys, v0s = _mixtures(F, shapes, seed=11, silent_f=4)
    mode = fca.FCA_FP64 if prec == "fp64" else fca.FCA_FP32_BULK
    ydev = [torch.from_numpy(y.astype(np.complex128) if prec == "fp64" else y).to(DEV) for y in ys]
    vdev = [torch.from_numpy(v.astype(np.float64) if prec == "fp64" else v).to(DEV) for v in v0s]
    ctx = fca.fca_init_batch(ydev, v0s=vdev, prec=mode)
    try:
        fca.fca_set_mask_covariances(ctx, sharpen=p, load=load)
        got = _start_R(fca, ctx)
        for k, (y, v0) in enumerate(zip(ys, v0s)):
            want = mask_init.mask_covariances(y.astype(np.complex128), v0.astype(np.float64), p, load)
            np.testing.assert_allclose(got[k], want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
            M = y.shape[2]
            np.testing.assert_allclose(got[k][:, 4], np.broadcast_to((1 + load) * np.eye(M), (2, M, M)),
                                       atol=1e-12)
        # a reset returns to the mask start; the powers are the given ones
        fca.fca_em_step(ctx, 3, want_loglik=False, want_R=False, want_v=False, allow_flags=True)
        fca.fca_reset(ctx)
        again = _start_R(fca, ctx)
        for a, b in zip(again, got):
            np.testing.assert_array_equal(a, b)
        _, _, v = fca.fca_em_step(ctx, 0, want_loglik=False, want_R=False, allow_flags=True)
        for vk, v0 in zip(v, v0s):
            np.testing.assert_array_equal(vk.cpu().numpy(), v0.astype(vk.cpu().numpy().dtype))
    finally:
        fca.fca_destroy(ctx)


def test_mask_start_subset_and_default_back(fca):
    """Listing one mixture changes only its start; fca_set_start without R0
    puts the default R back."""
    F = 5
    ys, v0s = _mixtures(F, [(4, 200), (4, 130), (3, 64)], seed=12)
    ctx = fca.fca_init_batch([torch.from_numpy(y).to(DEV) for y in ys],
                             v0s=[torch.from_numpy(v).to(DEV) for v in v0s])
    try:
        fca.fca_set_mask_covariances(ctx, mixtures=[1], sharpen=1.0, load=0.05)
        got = _start_R(fca, ctx)
        want = mask_init.mask_covariances(ys[1].astype(np.complex128), v0s[1].astype(np.float64), 1.0, 0.05)
        np.testing.assert_allclose(got[1], want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
        for k in (0, 2):
            M = ys[k].shape[2]
            np.testing.assert_allclose(got[k], _default_R(M, F), atol=1e-12)
        fca.fca_set_start(ctx, 1, v0=torch.from_numpy(v0s[1]).to(DEV))
        np.testing.assert_allclose(_start_R(fca, ctx)[1], _default_R(4, F), atol=1e-12)
    finally:
        fca.fca_destroy(ctx)


def test_mask_start_argument_errors(fca):
    ys, v0s = _mixtures(3, [(4, 50)], seed=13)
    ctx = fca.fca_init_batch([torch.from_numpy(ys[0]).to(DEV)])
    try:
        for kw in ({"sharpen": 0.5}, {"sharpen": 65.0}, {"load": 0.0}, {"load": -1.0}, {"load": float("nan")},
                   {"mixtures": [1]}, {"mixtures": [-1]}):
            with pytest.raises(fca.FcaError) as e:
                fca.fca_set_mask_covariances(ctx, **kw)
            assert e.value.status == fca.FCA_E_ARG
        # the plain start's equal powers would give R1 = R2 (a fixed point of the EM)
        with pytest.raises(fca.FcaError, match="equal powers") as e:
            fca.fca_set_mask_covariances(ctx)
        assert e.value.status == fca.FCA_E_ARG
        L = fca.lib()
        assert L.fca_set_mask_covariances(ctx.handle, 0, None, 3.0, 1e-3) == fca.FCA_E_ARG
        assert L.fca_set_mask_covariances(None, 1, None, 3.0, 1e-3) == fca.FCA_E_ARG
    finally:
        fca.fca_destroy(ctx)
