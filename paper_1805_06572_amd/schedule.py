"""Batched EM runs that stop each mixture on its own criterion.

All mixtures of a context advance together, `chunk` iterations per
fca_em_step call; after each call every mixture whose stopping rule holds is
taken out of later calls with fca_set_active, so the remaining mixtures get
the whole GPU.
"""
from __future__ import annotations

import numpy as np
import torch

from . import fca


def run_batch(ctx, max_iters: int, chunk, stop, weights=None):
    """Run until every mixture is stopped or has had max_iters iterations.

    chunk: iterations per fca_em_step call, an int or a sequence of ints whose
    last entry repeats (e.g. (16, 8, 4): few calls while no mixture can be
    done yet, fine steps later). stop(b, ll) -> bool is asked after every
    chunk with the log-likelihood
    history ll = [LL(theta^(0)), ..., LL(theta^(l-1))] of each still-active
    mixture b after l iterations (the parameters then stand at theta^(l), at
    least as likely by the monotonicity of EM).
    weights: optional [B, F] tensor on the context's device; the histories
    are then sum_f weights[b, f] LL_f (per-frequency values from
    fca_loglik_per_freq), e.g. a 0/1 mask of the frequencies a comparison
    trusts.
    Returns (iterations run per mixture [B], list of LL histories)."""
    B = ctx.B
    hist = [[] for _ in range(B)]
    iters = np.zeros(B, dtype=np.int64)
    active = np.ones(B, dtype=bool)
    chunks = [int(chunk)] if np.isscalar(chunk) else [int(c) for c in chunk]
    call = 0
    while active.any():
        k = int(min(chunks[min(call, len(chunks) - 1)], max_iters - iters[active].max()))
        call += 1
        if k <= 0:
            break
        ll, _, _ = fca.fca_em_step(ctx, k, want_loglik=weights is None, want_R=False, want_v=False,
                                   allow_flags=True)
        if weights is None:
            ll = ll.cpu().numpy()
        else:
            assert k <= 128, "per-frequency rows cover at most 128 iterations of a call"
            per_f = fca.fca_loglik_per_freq(ctx, k)                   # [k, B, F]
            per_f = torch.where(weights > 0, per_f * weights, torch.zeros_like(per_f))
            ll = per_f.sum(-1).T.cpu().numpy()                          # [B, k]
        for b in np.nonzero(active)[0]:
            hist[b].extend(ll[b].tolist())
            iters[b] += k
            if iters[b] >= max_iters or stop(int(b), hist[b]):
                active[b] = False
                fca.fca_set_active(ctx, int(b), False)
    for b in range(B):
        fca.fca_set_active(ctx, b, True)
    return iters, hist


def converged(rel_tol: float):
    """Stopping rule: the last iteration raised the log-likelihood by less
    than rel_tol times its total rise from LL(theta^(0))."""
    def stop(b, ll):
        if len(ll) < 3:
            return False
        return (ll[-1] - ll[-2]) <= rel_tol * abs(ll[-1] - ll[0])
    return stop


def reached(targets):
    """Stopping rule: the log-likelihood reached targets[b]."""
    def stop(b, ll):
        return ll[-1] >= targets[b]
    return stop
