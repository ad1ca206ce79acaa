"""Learned initial powers for the EM (optional; not part of the paper).

Trains the library's per-bin network (fca_mlp_*, hand-written HIP kernels)
on independent bins of the array workload, and produces the learned start
v_j^(0) = (r, 1 - r) 2 ||y||^2 / M for a mixture. The plain start stays the
fallback: `choose_starts` evaluates the log-likelihood of both starts with
the EM itself (after one iteration by default) and keeps the better one. The
learned powers can also serve as time-frequency masks for the initial
spatial covariances (fca_set_mask_covariances).
"""
from __future__ import annotations

import numpy as np
import torch

from . import fca, synth


def train(M: int = 4, F: int = 513, steps: int = 400, batch: int = 8192, lr: float = 1e-3,
          weight_decay: float = 1e-4, seed: int = 0, chunk_steps: int = 50, log=None, hidden: int = 256,
          cosine: bool = False):
    """Train a network of hidden width `hidden` for M microphones on
    independent bins drawn on the device (synth.array_bins_device), AdamW at
    rate lr (cosine: decayed to 0 over the steps); returns (Mlp, list of
    batch losses)."""
    net = fca.Mlp(M, seed=seed, max_batch=batch, hidden=hidden)
    g = torch.Generator(device=net.device).manual_seed(10_000 + seed)
    losses = []
    step = 0
    while step < steps:
        k = min(chunk_steps, steps - step)
        yt, ft, rt = synth.array_bins_device(k * batch, M, F, g, device=net.device)
        for i in range(k):
            sl = slice(i * batch, (i + 1) * batch)
            loss, _ = fca.fca_mlp_backward(net, yt[sl], ft[sl], rt[sl])
            t = step + i
            lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * t / steps)) if cosine else lr
            fca.fca_mlp_adamw(net, lr=lr_t, weight_decay=weight_decay)
            losses.append(loss)
        step += k
        if log:
            log(f"step {step}: loss {np.mean(losses[-k:]):.5f}")
    return net, losses


def evaluate(net, n: int = 65536, M: int = 4, F: int = 513, seed: int = 99):
    """(network loss, loss of the best constant predictor) on held-out bins."""
    from .fca import fca_mlp_forward
    rng = np.random.default_rng(20_000 + seed)
    y, fpos, r = synth.array_bins(n, M, F, rng)
    yt, ft = torch.from_numpy(y).cuda(), torch.from_numpy(fpos).cuda()
    pred = np.concatenate([fca_mlp_forward(net, yt[i:i + net.max_batch], ft[i:i + net.max_batch]).cpu().numpy()
                           for i in range(0, n, net.max_batch)])
    pred = np.clip(pred.astype(np.float64), 1e-7, 1 - 1e-7)
    t = r.astype(np.float64)
    bce = float(np.mean(-(t * np.log(pred) + (1 - t) * np.log(1 - pred))))
    c = t.mean()
    bce_const = float(np.mean(-(t * np.log(c) + (1 - t) * np.log(1 - c))))
    return bce, bce_const


def choose_starts(net, ctx, ys, choice_iter: int = 1, mask_sharpen=None, mask_load: float = 1e-3):
    """Per mixture of a batched FP32 context, keep whichever of the plain and
    the learned start has the higher log-likelihood after `choice_iter` EM
    iterations, LL(theta^choice_iter) (both evaluated by the EM itself, all
    mixtures in one batch per start). choice_iter = 0 compares the starts
    themselves; that favours the plain start, whose equal powers fit the
    mixture's total power well but leave the sources undistinguished, while
    one iteration is enough to show the learned start ahead.

    With mask_sharpen set, the learned start also takes its spatial
    covariances from the network's masks (fca_set_mask_covariances with
    that sharpening and mask_load); the plain start keeps the default R.
    That start is far ahead already at theta^0, so choice_iter = 0 suffices
    for it.

    Expects ctx fresh, at its plain starts. The learned run is not thrown
    away: a mixture that keeps its learned start stays at
    theta^(choice_iter + 1) of it; a mixture that falls back is reset to its
    plain theta^0. Returns (chosen [B] bool: learned start kept, ll_plain [B],
    ll_learned [B], advanced [B]: EM iterations already run from the chosen
    start)."""
    # the plain run is thrown away: j iterations, then an evaluation-only pass
    # for LL(theta^j)
    if choice_iter > 0:
        fca.fca_em_step(ctx, choice_iter, want_loglik=False, want_R=False, want_v=False, allow_flags=True)
    ll, _, _ = fca.fca_em_step(ctx, 0, want_R=False, want_v=False, allow_flags=True)
    ll_plain = ll[:, 0].cpu().numpy()
    fca.fca_set_learned_starts(ctx, net)
    if mask_sharpen is not None:
        fca.fca_set_mask_covariances(ctx, sharpen=mask_sharpen, load=mask_load)
    ll, _, _ = fca.fca_em_step(ctx, choice_iter + 1, want_R=False, want_v=False, allow_flags=True)
    ll_learned = ll[:, choice_iter].cpu().numpy()
    chosen = ll_learned > ll_plain
    for b in np.nonzero(~chosen)[0]:
        fca.fca_set_start(ctx, int(b))
    advanced = np.where(chosen, choice_iter + 1, 0)
    return chosen, ll_plain, ll_learned, advanced


def choose_start(net, y: torch.Tensor):
    """(v0 or None, ll_plain, ll_learned): the learned start if the EM rates it
    higher than the plain start at iteration 0, else None (plain start)."""
    v0 = fca.fca_mlp_init_powers(net, y)
    lls = []
    for start in (None, v0):
        ctx = fca.fca_init(y, v0=start, prec=fca.FCA_FP32_BULK)
        try:
            ll, _, _ = fca.fca_em_step(ctx, 0, want_R=False, want_v=False, allow_flags=True)
        finally:
            fca.fca_destroy(ctx)
        lls.append(float(ll.cpu().numpy()[0, 0]))
    return (v0 if lls[1] > lls[0] else None), lls[0], lls[1]
