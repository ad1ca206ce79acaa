"""More than two sources -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module; the product path never does.

The paper's model (Section 2) with J >= 2 sources, y = sum_j x_j,
x_j ~ CN(0, v_j S_j), and two EMs for it, plain FP64 numpy with loops over
frequencies and frames:

exact_em  the conventional EM (Section 2 with the sums over all J sources):
          R = sum_k v_k S_k, mu_j = v_j S_j R^-1 y,
          Phi_j = mu_j mu_j^H + v_j S_j - v_j S_j R^-1 v_j S_j (the posterior
          covariance of x_j; for J = 2 it is eq. postquadexp),
          v_j' = tr(S_j^-1 Phi_j) / M (old S_j), S_j' = mean_n Phi_j / v_j'.

fast_em   the reading of the paper's future work built by the library:
          parameters S_j = P^-H Lambda_j P^-1 with one basis P per frequency
          (Lambda_J = I), the E-step and power update in that basis (exact
          for such parameters), then the new S~_j = P^H S_j' P projected
          back onto that form by approximate joint diagonalisation (ajd):
          whitening by S~_J and a unitary Jacobi AJD of the others with the
          Cardoso-Souloumiac angles, in sweeps of rounds x = 1 .. MP-1 that
          rotate the disjoint pairs (k, k XOR x). For J = 2 the AJD is the
          exact eigendecomposition and fast_em is FastFCA (Algorithm 1).

Layouts: y [F, N, M]; S [J, F, M, M]; v [J, F, N]; ll [iters + 1, F].
"""
from __future__ import annotations

import numpy as np

MAX_SWEEPS = 16


def herm(A):
    return np.conj(np.swapaxes(A, -1, -2))


# ------------------------------------------------------------------ exact EM
def exact_em(y, S0, v0, iters):
    """Conventional J-source EM. Returns (S, v, ll) with ll[l, f] the
    log-likelihood of theta^(l)."""
    y = np.asarray(y, dtype=np.complex128)
    F, N, M = y.shape
    S = np.array(S0, dtype=np.complex128)
    v = np.array(v0, dtype=np.float64)
    J = S.shape[0]
    ll = np.zeros((iters + 1, F))
    for l in range(iters + 1):
        Sn = np.zeros_like(S)
        vn = np.zeros_like(v)
        for f in range(F):
            Sinv = [np.linalg.inv(S[j, f]) for j in range(J)]
            Phis = [[] for _ in range(J)]
            for n in range(N):
                Rj = [v[j, f, n] * S[j, f] for j in range(J)]
                R = sum(Rj)
                yy = y[f, n]
                Ri_y = np.linalg.solve(R, yy)
                sign, logdet = np.linalg.slogdet(R)
                ll[l, f] += -M * np.log(np.pi) - logdet - np.real(np.vdot(yy, Ri_y))
                for j in range(J):
                    mu = Rj[j] @ Ri_y
                    post = Rj[j] - Rj[j] @ np.linalg.solve(R, Rj[j])
                    post = 0.5 * (post + herm(post))
                    Phi = np.outer(mu, np.conj(mu)) + post
                    Phis[j].append(Phi)
                    vn[j, f, n] = np.real(np.trace(Sinv[j] @ Phi)) / M
            for j in range(J):
                A = sum(Phis[j][n] / vn[j, f, n] for n in range(N)) / N
                Sn[j, f] = 0.5 * (A + herm(A))
        if l < iters:
            S, v = Sn, vn
    return S, v, ll


# ------------------------------------------------------------------ AJD
def cs_rotation(Cs, p, q):
    """(c, s) of the Cardoso-Souloumiac rotation of the pair (p, q) for the
    Hermitian matrices Cs. With s = sin(t) exp(i phi), c = cos(t), the
    rotated C'_pp - C'_qq = w . h with w = (cos 2t, sin 2t cos phi,
    sin 2t sin phi) and h = (C_pp - C_qq, 2 Re C_pq, -2 Im C_pq); the unit
    dominant eigenvector (x, y, z), x >= 0, of G = sum_j h_j h_j^T maximises
    sum_j (C'_j,pp - C'_j,qq)^2, i.e. minimises the rotated off-diagonal
    entries, and gives c = sqrt((1 + x) / 2), s = (y + i z) / (2 c)."""
    G = np.zeros((3, 3))
    for C in Cs:
        h = np.array([np.real(C[p, p] - C[q, q]), 2 * np.real(C[p, q]), -2 * np.imag(C[p, q])])
        G += np.outer(h, h)
    w, V = np.linalg.eigh(G)
    x, yv, z = V[:, -1]
    if x < 0:
        x, yv, z = -x, -yv, -z
    c = np.sqrt((1 + x) / 2)
    s = (yv + 1j * z) / (2 * c)
    return c, s


def rotate(A, p, q, c, s):
    """G^H A G for the rotation G_pp = G_qq = c, G_pq = -conj(s), G_qp = s."""
    G = np.eye(A.shape[0], dtype=np.complex128)
    G[p, p] = G[q, q] = c
    G[p, q] = -np.conj(s)
    G[q, p] = s
    return herm(G) @ A @ G, G


def ajd(Cs, tol):
    """Unitary Jacobi AJD of the Hermitian matrices Cs (list of M x M).
    Returns (U, rotated matrices, sweeps run). A pair is left alone when its
    off-diagonal entries are already small, sum_j |C_j,pq|^2 <= tol^2
    sum_j |C_j,pp C_j,qq|, or its rotation is tiny, |s| <= tol; sweeps stop
    after one without a rotation."""
    Cs = [np.array(C, dtype=np.complex128) for C in Cs]
    M = Cs[0].shape[0]
    MP = 1
    while MP < M:
        MP *= 2
    U = np.eye(M, dtype=np.complex128)
    sweeps = 0
    for sweeps in range(1, MAX_SWEEPS + 1):
        rotated = False
        for x in range(1, MP):
            for k in range(MP):
                p, q = k, k ^ x
                if not (p < q < M):
                    continue
                off = sum(abs(C[p, q]) ** 2 for C in Cs)
                if off <= tol * tol * sum(abs(np.real(C[p, p] * C[q, q])) for C in Cs):
                    continue
                c, s = cs_rotation(Cs, p, q)
                if abs(s) <= tol:
                    continue
                rotated = True
                for j in range(len(Cs)):
                    Cs[j], G = rotate(Cs[j], p, q, c, s)
                U = U @ G
        if not rotated:
            break
    return U, Cs, sweeps


def project(St, tol):
    """(Q, lam [J, M], log det S~_J) with Q^H S~_J Q = I and
    lam_j = diag(Q^H S~_j Q) by whitening with S~_J and ajd of the others."""
    J, M = St.shape[0], St.shape[1]
    L = np.linalg.cholesky(St[-1])
    Li = np.linalg.inv(L)
    Cs = [Li @ St[j] @ herm(Li) for j in range(J - 1)]
    U, Cr, _ = ajd(Cs, tol) if J > 1 else (np.eye(M), [], 0)
    Q = herm(Li) @ U
    lam = np.ones((J, M))
    for j in range(J - 1):
        lam[j] = np.real(np.diag(Cr[j]))
    logdet = 2 * np.sum(np.log(np.real(np.diag(L))))
    return Q, lam, logdet


# ------------------------------------------------------------------ AJD EM
def fast_em(y, S0, v0, iters, tol=1e-15):
    """The AJD method from S0 [J, F, M, M] (projected onto the jointly
    diagonalisable form first) and v0 [J, F, N]. Returns (S, v, ll, P, lam)
    with S_j = P^-H Lambda_j P^-1 of the final parameters and ll[l, f] the
    log-likelihood of theta^(l)."""
    y = np.asarray(y, dtype=np.complex128)
    F, N, M = y.shape
    S0 = np.asarray(S0, dtype=np.complex128)
    J = S0.shape[0]
    v = np.array(v0, dtype=np.float64)
    P = np.zeros((F, M, M), dtype=np.complex128)
    lam = np.zeros((F, J, M))
    logdetP = np.zeros(F)
    for f in range(F):
        P[f], lam[f], ld = project(S0[:, f], tol)
        logdetP[f] = -ld
    ll = np.zeros((iters + 1, F))
    for l in range(iters + 1):
        vn = np.zeros_like(v)
        for f in range(F):
            St = np.zeros((J, M, M), dtype=np.complex128)
            for n in range(N):
                yt = herm(P[f]) @ y[f, n]
                e = np.abs(yt) ** 2
                pw = v[:, f, n][:, None] * lam[f]          # [J, M]: v_j lam_ji
                d = pw.sum(0)
                ll[l, f] += -M * np.log(np.pi) + logdetP[f] - np.sum(np.log(d)) - np.sum(e / d)
                for j in range(J):
                    mu = pw[j] * yt / d
                    c = pw[j] * (d - pw[j]) / d
                    vn[j, f, n] = np.sum((np.abs(mu) ** 2 + c) / lam[f, j]) / M
                    St[j] += (np.outer(mu, np.conj(mu)) + np.diag(c)) / vn[j, f, n]
            if l < iters:
                St = St / N
                St = 0.5 * (St + herm(St))
                Q, lam[f], ld = project(St, tol)
                P[f] = P[f] @ Q
                logdetP[f] -= ld
        if l < iters:
            v = vn
    S = np.zeros((J, F, M, M), dtype=np.complex128)
    for f in range(F):
        Pi = np.linalg.inv(P[f])
        for j in range(J):
            S[j, f] = herm(Pi) @ np.diag(lam[f, j]) @ Pi
    return S, v, ll, P, lam


def mmse(y, P, lam, v):
    """x [J, F, N, M]: mu_j = P^-H mu~_j in the basis form."""
    y = np.asarray(y, dtype=np.complex128)
    F, N, M = y.shape
    J = lam.shape[1]
    x = np.zeros((J, F, N, M), dtype=np.complex128)
    for f in range(F):
        PiH = herm(np.linalg.inv(P[f]))
        for n in range(N):
            yt = herm(P[f]) @ y[f, n]
            pw = v[:, f, n][:, None] * lam[f]
            d = pw.sum(0)
            for j in range(J):
                x[j, f, n] = PiH @ (pw[j] * yt / d)
    return x


def default_start(y, J):
    """Plain start for J sources: S_j = I + 0.5 (j - 1) / (J - 1) e1 e1^H
    (J = 2: R1 = I, R2 = I + 0.5 e1 e1^H), v_j = ||y||^2 / M floored at 1e-12
    times its mean (1 if the mean is 0)."""
    y = np.asarray(y, dtype=np.complex128)
    F, N, M = y.shape
    S = np.zeros((J, F, M, M), dtype=np.complex128)
    for j in range(J):
        S[j] = np.eye(M)
        S[j, :, 0, 0] += 0.5 * j / (J - 1)
    p = np.sum(np.abs(y) ** 2, axis=-1) / M
    mean = p.mean()
    fl = 1e-12 * mean if mean > 0 else 1.0
    v = np.broadcast_to(np.maximum(p, fl), (J, F, N)).copy()
    return S, v
