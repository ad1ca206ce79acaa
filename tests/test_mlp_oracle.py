"""Pins of the FP64 MLP reference (CPU): its analytic gradient against
central finite differences, GELU against its definition, and the feature
map on a hand-checked bin."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import mlp
from paper_1805_06572_amd import synth


def small_params(rng, H=256):
    n_par = H * 32 + H + 2 * (H * H + H) + H + 1
    p = rng.standard_normal(n_par) * 0.05
    Ws, bs, w4, b4 = mlp.unpack(p)
    assert [W.shape for W in Ws] == [(H, 32), (H, H), (H, H)] and w4.shape == (H,)
    return p


@pytest.mark.parametrize("H", [256, 64, 32])
def test_gradient_matches_finite_differences(H):
    rng = np.random.default_rng(0)
    p = small_params(rng, H)
    y, fpos, r = synth.array_bins(16, 4, 513, rng)
    X = mlp.features(y, fpos)
    L, g = mlp.loss_and_grad(p, X, r.astype(np.float64))
    idx = rng.choice(len(p), 40, replace=False)
    for i in idx:
        h = 1e-5
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, r) - mlp.loss(p - e, X, r)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_gelu_definition_and_derivative():
    x = np.linspace(-6, 6, 101)
    from scipy.stats import norm
    np.testing.assert_allclose(mlp.gelu(x), x * norm.cdf(x), rtol=1e-12, atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def test_features_of_a_hand_checked_bin():
    y = np.array([[1 + 1j, 2j, -3.0, 0.0]])
    X = mlp.features(y, np.array([0.25]))
    np.testing.assert_allclose(X[0, :3], np.log([2.0, 4.0, 9.0]), rtol=1e-12)
    # angle(2j) - angle(1+1j) = pi/4; angle(-3) - angle(1+1j) = 3pi/4; y_4 = 0 -> (0, 0)
    np.testing.assert_allclose(X[0, 4:10], [np.cos(np.pi / 4), np.sin(np.pi / 4), np.cos(3 * np.pi / 4),
                                            np.sin(3 * np.pi / 4), 0.0, 0.0], atol=1e-12)
    assert X[0, 10] == 0.25 and np.all(X[0, 11:] == 0)


def test_bf16_rounding_is_nearest_even():
    a = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.14159265], np.float32)
    b = mlp.bf16_round(a)
    np.testing.assert_array_equal(b[:3], [1.0, 1.0, 1.0 + 2 ** -6])
    assert abs(b[3] - 3.140625) < 1e-7


def test_parameter_count_names_one_width():
    for H in (32, 64, 128, 256):
        assert mlp.hidden_width(mlp.num_params(H)) == H
    with pytest.raises(ValueError):
        mlp.hidden_width(mlp.num_params(64) + 1)


def _two_unit_net(w2_00):
    """H = 2; inputs 3 (sin) and 4 (f/(F-1)). Pre-activations stay at or
    beyond +-16 (GELU(x) = x, GELU(-x) = 0 to 1e-50) and every value is an
    integer below 256 (exact in BF16) unless w2_00 is not."""
    H = 2
    W1 = np.zeros((H, 32))
    W1[0, 3], W1[0, 4], W1[1, 3] = 16.0, 32.0, -16.0
    b1 = np.array([0.0, 0.0])
    W2 = np.array([[w2_00, 0.0], [1.0, 0.0]])
    b2 = np.array([0.0, -64.0])
    W3 = np.array([[1.0, 0.0], [-1.0, 0.0]])
    b3 = np.array([0.0, 0.0])
    w4, b4 = np.array([0.125, 0.0]), np.array([-4.0])
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3, w4, b4])


def test_bf16_storage_reading():
    """bf16=True rounds the weight matrices and hidden values the kernels
    store in BF16: with every value exact in BF16 it equals the FP64 path;
    a weight 1 + 2^-10 (between two BF16 neighbours of 1) acts as 1."""
    y = np.array([[1.0, 1j]])                     # sin = 1
    X = mlp.features(y, np.array([0.5]))          # f/(F-1) = 1/2
    # layer 1: 16 + 16 = 32 and -16; layer 2: 32 w and 32 - 64 = -32; layer 3: 32 w, -32 w; z = 4 w - 4
    r_exact, (pres, _, z) = mlp.forward(_two_unit_net(1.0), X)
    r_b, (_, _, zb) = mlp.forward(_two_unit_net(1.0), X, bf16=True)
    np.testing.assert_allclose(pres[0][0], [32.0, -16.0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(z, [0.0], atol=1e-12)
    np.testing.assert_allclose(zb, z, atol=1e-12)
    _, (_, _, z_off) = mlp.forward(_two_unit_net(1.0 + 2.0 ** -10), X)
    _, (_, _, z_off_b) = mlp.forward(_two_unit_net(1.0 + 2.0 ** -10), X, bf16=True)
    np.testing.assert_allclose(z_off, [4.0 * 2.0 ** -10], atol=1e-12)
    np.testing.assert_allclose(z_off_b, [0.0], atol=1e-12)
