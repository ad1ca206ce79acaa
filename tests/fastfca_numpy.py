"""A second, independent CPU implementation used only to pin the oracle.

FastFCA as summarised in Algorithm 1 of the paper (Section 3), written with
numpy and scipy.linalg.eigh(a, b) (LAPACK's Hermitian-definite generalized
eigensolver) in FP64. The paper states that FastFCA and the conventional EM
of Section 2 produce identical iterates; the tests check the C oracle (the
conventional EM) against this module on that claim. Neither the GPU path nor
the oracle imports this file.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def _gevd(S1, S2):
    """lam ascending, P with P^H S2 P = I and S1 P = S2 P diag(lam) (eq. GEVD)."""
    lam, P = scipy.linalg.eigh(S1, S2)
    return lam, P


def fastfca(y: np.ndarray, S0: np.ndarray, v0: np.ndarray, iters: int):
    """Returns (S [2,F,M,M], v [2,F,N], ll [iters+1, F])."""
    F, N, M = y.shape
    P = np.empty((F, M, M), np.complex128)
    lam = np.empty((F, M))
    for f in range(F):                     # Algorithm 1, initial P^(0), Lambda^(0)
        lam[f], P[f] = _gevd(S0[0, f], S0[1, f])
    v1 = v0[0].copy()
    v2 = v0[1].copy()

    def loglik(P, lam, v1, v2):
        yt = np.einsum("fmi,fnm->fni", np.conj(P), y)           # eq. (tildey)
        d = v1[..., None] * lam[:, None, :] + v2[..., None]
        # v1 S1 + v2 S2 = P^-H diag(d) P^-1, so log det = sum log d - log|det P|^2
        _, logabsdet = np.linalg.slogdet(P)
        per_bin = (-M * np.log(np.pi) + 2.0 * logabsdet[:, None]
                   - np.sum(np.log(d), -1) - np.sum(np.abs(yt) ** 2 / d, -1))
        return per_bin.sum(-1)

    lls = []
    for _ in range(iters):
        lls.append(loglik(P, lam, v1, v2))
        yt = np.einsum("fmi,fnm->fni", np.conj(P), y)           # step: eq. (tildey)
        a = v1[..., None] * lam[:, None, :]
        b = v2[..., None] * np.ones_like(lam)[:, None, :]
        d = a + b
        mu1 = a / d * yt                                         # eq. (MMSEtilde)
        mu2 = b / d * yt
        c = a * b / d                                            # eq. (updatePhitildeeff) diagonal
        v1n = np.mean((np.abs(mu1) ** 2 + c) / lam[:, None, :], -1)   # eq. (updateveff)
        v2n = np.mean(np.abs(mu2) ** 2 + c, -1)
        St = []
        for mu, vn in ((mu1, v1n), (mu2, v2n)):                  # eq. (updateStildeeff)
            outer = np.einsum("fni,fnk->fik", mu / vn[..., None], np.conj(mu))
            diag = np.einsum("fni->fi", c / vn[..., None])
            Sj = (outer + diag[..., None] * np.eye(M)) / N
            St.append(0.5 * (Sj + np.conj(np.swapaxes(Sj, -1, -2))))
        for f in range(F):                                       # eqs. (updatePeff), (updateLambdaeff)
            sig, Q = _gevd(St[0][f], St[1][f])
            P[f] = P[f] @ Q
            lam[f] = sig
        v1, v2 = v1n, v2n
    lls.append(loglik(P, lam, v1, v2))

    Pinv = np.linalg.inv(P)                                      # S_j from P, Lambda (eq. recoverS)
    S2 = np.conj(np.swapaxes(Pinv, -1, -2)) @ Pinv
    S1 = np.conj(np.swapaxes(Pinv, -1, -2)) @ (lam[..., None] * Pinv)
    S = np.stack([S1, S2])
    return S, np.stack([v1, v2]), np.stack(lls)
