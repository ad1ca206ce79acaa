"""Pins of the mask-based initial covariances of the oracle (oracle/mask_init.py).

The paper states that its experiments start from spatial covariances
estimated with time-frequency masks (Section 4) without a formula; the
oracle takes the mask-weighted covariance, normalised to trace M and loaded.
These checks tie it to an independent route (a QR factorisation of the
selected frames), to closed forms and to its symmetries."""
import numpy as np
import pytest

from oracle import mask_init


def _y(rng, F, N, M):
    return rng.standard_normal((F, N, M)) + 1j * rng.standard_normal((F, N, M))


def test_hard_masks_equal_gram_matrix_by_qr():
    """With 0/1 masks A_1 is the Gram matrix of the selected frames:
    A = Z^H Z for Z = conj(Y_S), which a QR factorisation gives as T^H T."""
    rng = np.random.default_rng(0)
    F, N, M, load = 3, 40, 4, 1e-3
    y = _y(rng, F, N, M)
    sel = rng.random((F, N)) < 0.4
    v0 = np.stack([sel.astype(float), (~sel).astype(float)])
    R = mask_init.mask_covariances(y, v0, sharpen=3.0, load=load)
    for f in range(F):
        for j, s in enumerate((sel[f], ~sel[f])):
            _, T = np.linalg.qr(np.conj(y[f, s]))
            A = T.conj().T @ T
            want = M * A / np.trace(A).real + load * np.eye(M)
            np.testing.assert_allclose(R[j, f], want, rtol=1e-12, atol=1e-12)


def test_trace_hermitian_positive_definite():
    rng = np.random.default_rng(1)
    F, N, M, load = 4, 30, 3, 1e-2
    y = _y(rng, F, N, M)
    v0 = rng.gamma(0.5, 1.0, size=(2, F, N))
    R = mask_init.mask_covariances(y, v0, sharpen=2.0, load=load)
    np.testing.assert_allclose(np.trace(R, axis1=-2, axis2=-1).real, M * (1 + load), rtol=1e-13)
    np.testing.assert_allclose(R, np.conj(np.swapaxes(R, -1, -2)), atol=1e-14)
    assert np.all(np.linalg.eigvalsh(R) > 0)


def test_invariances_and_source_swap():
    """Scaling the powers or the mixture leaves R unchanged; swapping the
    sources swaps R_1 and R_2."""
    rng = np.random.default_rng(2)
    F, N, M = 3, 25, 4
    y = _y(rng, F, N, M)
    v0 = rng.gamma(0.5, 1.0, size=(2, F, N))
    R = mask_init.mask_covariances(y, v0)
    np.testing.assert_allclose(mask_init.mask_covariances(y, 7.5 * v0), R, rtol=1e-12)
    np.testing.assert_allclose(mask_init.mask_covariances((2 - 3j) * y, v0), R, rtol=1e-12)
    np.testing.assert_allclose(mask_init.mask_covariances(y, v0[::-1]), R[::-1], rtol=1e-12)


def test_equal_powers_give_the_sample_covariance_for_both_sources():
    rng = np.random.default_rng(3)
    F, N, M, load = 2, 50, 4, 1e-3
    y = _y(rng, F, N, M)
    v0 = np.ones((2, F, N))
    R = mask_init.mask_covariances(y, v0, sharpen=5.0, load=load)
    for f in range(F):
        C = np.cov(y[f].T, bias=True) + np.outer(y[f].mean(0), y[f].mean(0).conj())  # E[y y^H]
        np.testing.assert_allclose(R[0, f], M * C / np.trace(C).real + load * np.eye(M), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(R[0], R[1], rtol=1e-13)


def test_rank_one_mixture_and_silent_frequency():
    """y = s(n) a gives R_j = M a a^H / |a|^2 + load I whatever the masks; a
    silent frequency gives (1 + load) I."""
    rng = np.random.default_rng(4)
    F, N, M, load = 2, 20, 3, 0.1
    a = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    s = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    y = np.zeros((F, N, M), dtype=np.complex128)
    y[0] = s[:, None] * a[None, :]
    v0 = rng.gamma(0.5, 1.0, size=(2, F, N))
    R = mask_init.mask_covariances(y, v0, load=load)
    want = M * np.outer(a, a.conj()) / np.vdot(a, a).real + load * np.eye(M)
    np.testing.assert_allclose(R[:, 0], np.stack([want, want]), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(R[:, 1], np.broadcast_to((1 + load) * np.eye(M), (2, M, M)), atol=0)


@pytest.mark.parametrize("r,p", [(0.8, 3.0), (0.3, 2.0), (0.5, 7.0), (0.0, 3.0)])
def test_sharpened_mask_closed_form(r, p):
    v0 = np.array([[[r]], [[1.0 - r]]])
    w = mask_init.masks(v0, p)
    want = r ** p / (r ** p + (1 - r) ** p)
    np.testing.assert_allclose(w[:, 0, 0], [want, 1 - want], rtol=1e-15)
    # both powers zero: an even split
    np.testing.assert_array_equal(mask_init.masks(np.zeros((2, 1, 1)), p)[:, 0, 0], [0.5, 0.5])
