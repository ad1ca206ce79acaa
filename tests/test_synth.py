"""The device draw of training bins (synth.array_bins_device, run here on the
CPU) follows the same model as the numpy draw: moments that the model fixes
(E|y_m|^2 = 2 E[v] (1 + 0.1) with E[v] = exp(mu + sigma^2 / 2), the law of
r = v1 / (v1 + v2), uniform frequencies) and the spatial cross-moments."""
from __future__ import annotations

import numpy as np
import torch

from paper_1805_06572_amd import synth


def test_device_training_bins_match_the_model():
    n, M, F = 200_000, 4, 513
    y, fpos, r = synth.array_bins_device(n, M, F, torch.Generator().manual_seed(1), device="cpu")
    y, fpos, r = y.numpy(), fpos.numpy(), r.numpy()
    y2, fpos2, r2 = synth.array_bins(n, M, F, np.random.default_rng(1))
    assert y.shape == (n, M) and y.dtype == np.complex64
    assert fpos.min() >= 0 and fpos.max() <= 1 and np.all((r > 0) & (r < 1))
    ev = np.exp(-1.9635100260214235 + np.pi ** 2 / 4)       # E[v] of the log-normal powers
    want = 2 * ev * 1.1
    # heavy-tailed powers: the sample mean of 2e5 bins is within a few percent
    assert abs((np.abs(y) ** 2).mean() / want - 1) < 0.06
    assert abs((np.abs(y2) ** 2).mean() / want - 1) < 0.06
    assert abs(r.mean() - 0.5) < 0.005 and abs(r.std() - r2.std()) < 0.005
    assert abs(fpos.mean() - 0.5) < 0.005
    for i, j in ((1, 0), (3, 0), (2, 1)):
        a = np.abs(y[:, i] * np.conj(y[:, j])).mean()
        b = np.abs(y2[:, i] * np.conj(y2[:, j])).mean()
        assert abs(a / b - 1) < 0.06
