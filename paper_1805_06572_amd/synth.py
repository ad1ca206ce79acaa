"""Seeded synthetic multichannel STFT mixtures for the two-source full-rank
spatial covariance model (Section 2 of the FastFCA paper): y = x1 + x2 with
x_j(n,f) ~ CN(0, v_j(n,f) R_j(f)), R_j Hermitian positive definite and v_j > 0.

This module only draws inputs. It holds none of the EM arithmetic and is the
one piece shared by the CPU oracle tests, the GPU tests and the benchmark.
All arrays use the layout y[f, n, m], R[j, f, m, m'], v[j, f, n],
x[j, f, n, m]; complex Gaussian means E[z z^H] = I with z = (a + ib)/sqrt(2).

Workloads
---------
* ``random``  : R_j(f) = A A^H + 0.1 I with A an M x M matrix of i.i.d.
  CN(0,1) entries drawn independently per source and frequency;
  v_j(n,f) ~ Gamma(shape 0.5, scale 1) i.i.d.; complex128.
* ``array``   : a uniform linear array (spacing 4 cm, c = 343 m/s,
  fs = 16 kHz). R_j(f) = a_j(f) a_j(f)^H + 0.1 Gamma(f), with a_j the
  steering vector of a direction of arrival drawn uniformly in [0, pi)
  once per source, and Gamma(f) the spherically isotropic (sinc) diffuse
  coherence. Bin k sits at k * fs / (2 (F - 1)) Hz. y is rounded to
  complex64 when ``complex64=True``.
The paper's own data (speech convolved with measured room responses) is not
available; these draws stand in for it with the paper's STFT shape (F = 513
bins of a 1024-point frame at 16 kHz).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FS_HZ = 16000.0
MIC_SPACING_M = 0.04
SOUND_SPEED_MPS = 343.0


def cn(rng: np.random.Generator, shape) -> np.ndarray:
    """Standard circular complex Gaussian CN(0, 1) samples."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


@dataclass
class Mixture:
    y: np.ndarray        # [F, N, M] complex observed mixture
    R: np.ndarray        # [2, F, M, M] true spatial covariances
    v: np.ndarray        # [2, F, N] true source powers
    x: np.ndarray        # [2, F, N, M] true source images
    theta: np.ndarray | None = None  # DOAs of the array workload (radians)

    @property
    def shape(self):
        F, N, M = self.y.shape
        return M, F, N


def bin_frequencies_hz(F: int, fs: float = FS_HZ) -> np.ndarray:
    """Centre frequency of STFT bins 0..F-1 (DC .. Nyquist inclusive)."""
    if F == 1:
        return np.zeros(1)
    return np.arange(F) * fs / (2.0 * (F - 1))


def steering_vectors(theta: float, M: int, F: int, d: float = MIC_SPACING_M,
                     c: float = SOUND_SPEED_MPS, fs: float = FS_HZ) -> np.ndarray:
    """[F, M] far-field ULA steering vectors, microphone 1 as phase reference."""
    fhz = bin_frequencies_hz(F, fs)
    m = np.arange(M)
    return np.exp(-2j * np.pi * fhz[:, None] * m[None, :] * d * np.cos(theta) / c)


def diffuse_coherence(M: int, F: int, d: float = MIC_SPACING_M,
                      c: float = SOUND_SPEED_MPS, fs: float = FS_HZ) -> np.ndarray:
    """[F, M, M] spherically isotropic coherence sin(x)/x, x = 2 pi f |m-m'| d / c."""
    fhz = bin_frequencies_hz(F, fs)
    dist = np.abs(np.arange(M)[:, None] - np.arange(M)[None, :]) * d
    arg = 2.0 * np.pi * fhz[:, None, None] * dist[None, :, :] / c
    return np.sinc(arg / np.pi)  # numpy sinc is sin(pi x)/(pi x)


def random_covariances(rng: np.random.Generator, M: int, F: int) -> np.ndarray:
    A = cn(rng, (2, F, M, M))
    return A @ np.conj(np.swapaxes(A, -1, -2)) + 0.1 * np.eye(M)


def array_covariances(theta: np.ndarray, M: int, F: int) -> np.ndarray:
    G = diffuse_coherence(M, F)
    R = np.empty((2, F, M, M), dtype=np.complex128)
    for j in range(2):
        a = steering_vectors(float(theta[j]), M, F)
        R[j] = a[:, :, None] * np.conj(a[:, None, :]) + 0.1 * G
    return R


def _sqrt_factor(R: np.ndarray, method: str) -> np.ndarray:
    """A factor B with B B^H = R (Cholesky, or the PSD eigen square root)."""
    if method == "chol":
        return np.linalg.cholesky(R)
    w, U = np.linalg.eigh(R)
    return U * np.sqrt(np.clip(w, 0.0, None))[..., None, :]


def draw_images(R: np.ndarray, v: np.ndarray, z: np.ndarray, method: str) -> np.ndarray:
    """x_j(n,f) = sqrt(v_j(n,f)) B_j(f) z_j(n,f) so that E[x x^H] = v_j R_j."""
    B = _sqrt_factor(R, method)                       # [2, F, M, M]
    x = np.einsum("jfab,jfnb->jfna", B, z)
    return x * np.sqrt(v)[..., None]


def random_mixture(M: int = 2, F: int = 257, N: int = 200, seed: int = 0) -> Mixture:
    """The ``random`` workload. Draw order: A, then v, then z."""
    rng = np.random.default_rng(seed)
    R = random_covariances(rng, M, F)
    v = rng.gamma(0.5, 1.0, size=(2, F, N))
    z = cn(rng, (2, F, N, M))
    x = draw_images(R, v, z, "chol")
    return Mixture(y=x[0] + x[1], R=R, v=v, x=x)


def array_mixture(M: int = 4, F: int = 513, N: int = 1000, seed: int = 1,
                  complex64: bool = True, v: np.ndarray | None = None) -> Mixture:
    """The ``array`` workload. Draw order: both DOAs, then v, then z.

    ``v`` may be supplied (e.g. a temporally correlated draw); it is then
    used instead of the Gamma draw, and the DOAs and z are drawn as usual.
    """
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, np.pi, size=2)
    R = array_covariances(theta, M, F)
    vg = rng.gamma(0.5, 1.0, size=(2, F, N))
    if v is None:
        v = vg
    z = cn(rng, (2, F, N, M))
    x = draw_images(R, v, z, "eig")
    y = x[0] + x[1]
    if complex64:
        y = y.astype(np.complex64)
    return Mixture(y=y, R=R, v=v, x=x, theta=theta)


def ar1_log_powers(rng: np.random.Generator, F: int, N: int, rho: float = 0.9) -> np.ndarray:
    """[2, F, N] source powers whose logs follow a stationary AR(1) in n with
    coefficient rho, mean and variance matched to log Gamma(0.5, 1):
    E[log v] = digamma(0.5), Var[log v] = trigamma(0.5) = pi^2 / 2."""
    mu = -1.9635100260214235          # digamma(0.5) = -gamma - 2 log 2
    var = np.pi ** 2 / 2.0
    sd_e = np.sqrt(var * (1.0 - rho * rho))
    lv = np.empty((2, F, N))
    lv[:, :, 0] = mu + np.sqrt(var) * rng.standard_normal((2, F))
    e = sd_e * rng.standard_normal((2, F, N))
    for n in range(1, N):
        lv[:, :, n] = mu + rho * (lv[:, :, n - 1] - mu) + e[:, :, n]
    return np.exp(lv)


def array_bins(n: int, M: int, F: int, rng: np.random.Generator):
    """n independent time-frequency bins of the array workload, for training
    the learned initialisation. Each bin draws its own two DOAs (source 1 is
    the one with the smaller angle), its frequency bin uniformly in 0..F-1
    and its powers from the stationary marginal of the AR(1) log-power model
    (log-normal with the moments of log Gamma(0.5, 1)). The bins of one
    mixture share DOAs and are correlated in time; a per-bin network only sees
    one bin, whose marginal distribution is the same.
    Returns y [n, M] complex64, fpos [n] = f/(F-1) float32, r [n] = v1/(v1+v2)
    float32."""
    theta = np.sort(rng.uniform(0.0, np.pi, size=(n, 2)), axis=1)
    k = rng.integers(0, F, size=n)
    fhz = bin_frequencies_hz(F)[k]
    mu, var = -1.9635100260214235, np.pi ** 2 / 2.0
    v = np.exp(mu + np.sqrt(var) * rng.standard_normal((n, 2)))
    m = np.arange(M)
    dist = np.abs(m[:, None] - m[None, :]) * MIC_SPACING_M
    G = np.sinc(2.0 * fhz[:, None, None] * dist[None] / SOUND_SPEED_MPS)   # sin(x)/x, x = 2 pi f d / c
    z = cn(rng, (n, 2, M))
    y = np.zeros((n, M), np.complex128)
    for j in range(2):
        a = np.exp(-2j * np.pi * fhz[:, None] * m[None, :] * MIC_SPACING_M * np.cos(theta[:, j:j + 1])
                   / SOUND_SPEED_MPS)
        R = a[:, :, None] * np.conj(a[:, None, :]) + 0.1 * G
        w, U = np.linalg.eigh(R)
        B = U * np.sqrt(np.clip(w, 0.0, None))[:, None, :]
        y += np.sqrt(v[:, j])[:, None] * np.einsum("nab,nb->na", B, z[:, j])
    fpos = (k / max(F - 1, 1)).astype(np.float32)
    r = (v[:, 0] / (v[:, 0] + v[:, 1])).astype(np.float32)
    return y.astype(np.complex64), fpos, r


def array_bins_device(n: int, M: int, F: int, g, device="cuda:0"):
    """``array_bins`` drawn with torch on a device (the training batches of
    the learned start): the same model, drawn as x_j = sqrt(v_j) (a_j w_j +
    sqrt(0.1) Gamma(f)^(1/2) z_j) with w_j ~ CN(0, 1), z_j ~ CN(0, I), whose
    covariance is v_j (a_j a_j^H + 0.1 Gamma(f)) (Gamma's square root per
    frequency from its eigendecomposition, negative rounding clipped), and
    torch's generator g, so the draws differ from the numpy version.
    Returns device tensors y [n, M] complex64, fpos [n], r [n] float32."""
    import torch

    f32 = dict(device=device, dtype=torch.float32)
    fr = bin_frequencies_hz(F)
    mm = np.arange(M)
    dist = np.abs(mm[:, None] - mm[None, :]) * MIC_SPACING_M
    Gam = np.sinc(2.0 * fr[:, None, None] * dist[None] / SOUND_SPEED_MPS)     # [F, M, M] real
    w, U = np.linalg.eigh(Gam)
    BG = torch.from_numpy(U * np.sqrt(np.clip(w, 0.0, None))[:, None, :]).to(**f32)
    u = torch.rand((n, 2), generator=g, **f32) * float(np.pi)
    theta = torch.sort(u, dim=1).values                       # source 1: the smaller angle
    k = torch.randint(0, F, (n,), generator=g, device=device)
    fhz = torch.from_numpy(fr).to(**f32)[k]
    mu, var = -1.9635100260214235, np.pi ** 2 / 2.0
    v = torch.exp(mu + float(np.sqrt(var)) * torch.randn((n, 2), generator=g, **f32))
    m = torch.arange(M, **f32)
    y = torch.zeros((n, M), dtype=torch.complex64, device=device)

    def cn(shape):
        return torch.complex(torch.randn(shape, generator=g, **f32), torch.randn(shape, generator=g, **f32)) / float(
            np.sqrt(2.0))
    for j in range(2):
        ph = -2.0 * np.pi * fhz[:, None] * m[None, :] * MIC_SPACING_M * torch.cos(theta[:, j:j + 1]) / SOUND_SPEED_MPS
        a = torch.polar(torch.ones_like(ph), ph)                                 # [n, M]
        z = cn((n, M))
        Bk = BG[k]                                                              # [n, M, M] real
        diffuse = torch.complex((Bk * z.real[:, None, :]).sum(-1), (Bk * z.imag[:, None, :]).sum(-1))
        y = y + torch.sqrt(v[:, j])[:, None] * (a * cn((n, 1)) + float(np.sqrt(0.1)) * diffuse)
    fpos = k.to(torch.float32) / max(F - 1, 1)
    r = v[:, 0] / (v[:, 0] + v[:, 1])
    return y, fpos, r


def condition_numbers(R: np.ndarray) -> np.ndarray:
    """[F] max_j cond_2(R_j(f)) of the true covariances (a data property used
    to decide which bins a finite-precision comparison is meaningful on)."""
    w = np.linalg.eigvalsh(R)                         # [2, F, M] ascending
    with np.errstate(divide="ignore"):
        k = w[..., -1] / np.where(w[..., 0] > 0, w[..., 0], 0.0)
    return np.max(k, axis=0)


def default_initial_covariances(M: int, F: int) -> np.ndarray:
    """R1 = I and R2 = I + 0.5 e1 e1^H at every bin (the plain start)."""
    R0 = np.zeros((2, F, M, M), dtype=np.complex128)
    R0[:] = np.eye(M)
    R0[1, :, 0, 0] += 0.5
    return R0


def array_mixture_device(M: int, F: int, N: int, seed: int, device="cuda:0", ar1: bool = False):
    """The array workload drawn with torch on a device (for multi-GB inputs).

    Same model as ``array_mixture`` (DOAs uniform in [0, pi), R_j = a a^H +
    0.1 Gamma(f), eigen square root, powers Gamma(0.5, 1) or, with ar1, the
    AR(1) log-powers of ``ar1_log_powers``), but torch's generator: the draws
    differ from the numpy version with the same seed. Returns (y [F, N, M]
    complex64 on the device, theta [2] numpy, R [2, F, M, M] numpy)."""
    import torch

    g = torch.Generator(device=device).manual_seed(int(seed))
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, np.pi, size=2)
    R = array_covariances(theta, M, F)
    w, U = np.linalg.eigh(R)
    B = torch.from_numpy(U * np.sqrt(np.clip(w, 0.0, None))[..., None, :]).to(device=device, dtype=torch.complex64)
    y = torch.zeros((F, N, M), dtype=torch.complex64, device=device)
    for j in range(2):
        if ar1:
            mu, var, rho = -1.9635100260214235, np.pi ** 2 / 2.0, 0.9
            # x_n = rho x_(n-1) + e_n, x_0 stationary: a doubling scan over n
            # (x_n <- x_n + rho^s x_(n-s) for s = 1, 2, 4, ...)
            x = torch.randn((F, N), generator=g, device=device) * float(np.sqrt(var * (1 - rho * rho)))
            x[:, 0] = float(np.sqrt(var)) * torch.randn((F,), generator=g, device=device)
            s = 1
            while s < N:
                x = torch.cat([x[:, :s], x[:, s:] + float(rho ** s) * x[:, :-s]], dim=1)
                s *= 2
            v = torch.exp(mu + x)
        else:
            v = torch._standard_gamma(torch.full((F, N), 0.5, device=device), generator=g)
        z = torch.complex(torch.randn((F, N, M), generator=g, device=device),
                          torch.randn((F, N, M), generator=g, device=device)) / float(np.sqrt(2.0))
        x = torch.matmul(z, B[j].transpose(-1, -2))       # x[f, n] = B_j(f) z[f, n]
        y += x * torch.sqrt(v).unsqueeze(-1)
    return y, theta, R
