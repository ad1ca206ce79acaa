"""Thin ctypes binding of libfca.so (include/fca.h), same names as the C ABI.

Argument marshalling only: every step of the EM runs in the library's HIP
kernels; torch provides device memory and the stream. Inputs are torch
tensors (device or host) or numpy arrays; outputs are allocated as torch
tensors on the device of the input mixture. Loading fails loudly if the
library has not been built (``python -m paper_1805_06572_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfca.so")

FCA_OK = 0
FCA_E_ARG = -1
FCA_E_NOMEM = -2
FCA_E_DEVICE = -3
FCA_E_NOT_PD = -4
FCA_E_NONFINITE = -5
FCA_E_STATE = -6
FCA_FP64 = 0
FCA_FP32_BULK = 1
FCA_FLAG_NOT_PD = 1
FCA_FLAG_NONFINITE = 2
FCA_FLAG_SWEEPS = 4
STATUS_NAMES = {0: "FCA_OK", -1: "FCA_E_ARG", -2: "FCA_E_NOMEM", -3: "FCA_E_DEVICE",
                -4: "FCA_E_NOT_PD", -5: "FCA_E_NONFINITE", -6: "FCA_E_STATE"}

EXPORTED = ["fca_init", "fca_init_batch", "fca_reset", "fca_set_start", "fca_set_active", "fca_em_step", "fca_conv_em_step", "fca_separate",
            "fca_status_per_freq", "fca_last_error", "fca_destroy", "fca_gevd", "fca_timing",
            "fca_launch_groups", "fca_set_launch_shape", "fca_autotune", "fca_graph_capture", "fca_graph_launch",
            "fca_mlp_create", "fca_mlp_destroy", "fca_mlp_num_params", "fca_mlp_last_error",
            "fca_mlp_get_params", "fca_mlp_set_params", "fca_mlp_forward", "fca_mlp_backward",
            "fca_mlp_adamw", "fca_mlp_init_powers", "fca_mlp_init_powers_batch", "fca_set_learned_starts",
            "fca_set_mask_covariances", "fca_loglik_per_freq", "fca_em_solve_noalloc", "fca_stft", "fca_istft",
            "fca_stft_frames", "fca_multi_init", "fca_multi_em_step", "fca_multi_separate", "fca_multi_timing",
            "fca_multi_last_error", "fca_multi_destroy"]


class fca_problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("F", ctypes.c_int32), ("N", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("y", ctypes.c_void_p), ("y_stride_f", ctypes.c_int64),
                ("y_stride_n", ctypes.c_int64), ("y_stride_m", ctypes.c_int64),
                ("R0", ctypes.c_void_p), ("v0", ctypes.c_void_p), ("stream", ctypes.c_void_p)]


class FcaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libfca.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "`python -m paper_1805_06572_amd.build` (there is no fallback path)")
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.fca_init.argtypes = [ctypes.POINTER(fca_problem), ctypes.POINTER(vp)]
        L.fca_init_batch.argtypes = [ctypes.POINTER(fca_problem), i32, ctypes.POINTER(vp)]
        L.fca_reset.argtypes = [vp]
        L.fca_set_start.argtypes = [vp, i32, vp, vp]
        L.fca_set_active.argtypes = [vp, i32, i32]
        L.fca_em_step.argtypes = [vp, i32, vp, vp, vp]
        L.fca_conv_em_step.argtypes = [vp, i32, vp, vp, vp]
        L.fca_separate.argtypes = [vp, vp]
        L.fca_status_per_freq.argtypes = [vp, vp]
        L.fca_last_error.argtypes = [vp]
        L.fca_last_error.restype = ctypes.c_char_p
        L.fca_destroy.argtypes = [vp]
        L.fca_destroy.restype = None
        L.fca_gevd.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp]
        L.fca_timing.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.fca_launch_groups.argtypes = [vp, vp, i32, ctypes.POINTER(i32)]
        L.fca_set_launch_shape.argtypes = [vp, i32, i32, i32]
        L.fca_autotune.argtypes = [vp, i32]
        L.fca_graph_capture.argtypes = [vp, i32, i32, vp, vp, vp, vp]
        L.fca_graph_launch.argtypes = [vp, i32]
        L.fca_mlp_create.argtypes = [i32, i32, ctypes.c_uint64, i32, vp, ctypes.POINTER(vp)]
        L.fca_mlp_destroy.argtypes = [vp]
        L.fca_mlp_destroy.restype = None
        L.fca_mlp_num_params.argtypes = [vp]
        L.fca_mlp_num_params.restype = i64
        L.fca_mlp_last_error.argtypes = [vp]
        L.fca_mlp_last_error.restype = ctypes.c_char_p
        L.fca_mlp_get_params.argtypes = [vp, vp]
        L.fca_mlp_set_params.argtypes = [vp, vp]
        L.fca_mlp_forward.argtypes = [vp, vp, vp, i32, vp]
        L.fca_mlp_backward.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(ctypes.c_double), vp]
        L.fca_mlp_adamw.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float]
        L.fca_mlp_init_powers.argtypes = [vp, vp, i32, i32, vp]
        L.fca_mlp_init_powers_batch.argtypes = [vp, i32, ctypes.POINTER(vp), i32, ctypes.POINTER(i32),
                                                ctypes.POINTER(vp)]
        L.fca_set_learned_starts.argtypes = [vp, vp, i32, ctypes.POINTER(i32)]
        L.fca_set_mask_covariances.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.c_double, ctypes.c_double]
        L.fca_loglik_per_freq.argtypes = [vp, i32, vp]
        L.fca_em_solve_noalloc.argtypes = [i32, i32, i32, i32, vp, i64, vp, i32, i32, vp, vp, vp, vp]
        L.fca_stft_frames.argtypes = [i64, i32]
        L.fca_stft_frames.restype = i64
        L.fca_stft.argtypes = [i32, i64, i32, i32, vp, vp, vp]
        L.fca_istft.argtypes = [i32, i64, i32, i32, vp, vp, vp]
        L.fca_multi_init.argtypes = [ctypes.POINTER(fca_problem), i32, vp, vp, ctypes.POINTER(vp)]
        L.fca_multi_em_step.argtypes = [vp, i32, vp, vp, vp]
        L.fca_multi_separate.argtypes = [vp, vp]
        L.fca_multi_timing.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.fca_multi_last_error.argtypes = [vp]
        L.fca_multi_last_error.restype = ctypes.c_char_p
        L.fca_multi_destroy.argtypes = [vp]
        L.fca_multi_destroy.restype = None
        for name in ("fca_init", "fca_init_batch", "fca_reset", "fca_set_start", "fca_set_active", "fca_em_step", "fca_conv_em_step", "fca_separate",
                     "fca_status_per_freq", "fca_gevd", "fca_timing", "fca_launch_groups",
                     "fca_set_launch_shape", "fca_autotune", "fca_graph_capture", "fca_graph_launch", "fca_mlp_create", "fca_mlp_get_params",
                     "fca_mlp_set_params", "fca_mlp_forward", "fca_mlp_backward", "fca_mlp_adamw",
                     "fca_mlp_init_powers", "fca_mlp_init_powers_batch", "fca_set_learned_starts",
                     "fca_set_mask_covariances", "fca_loglik_per_freq", "fca_em_solve_noalloc", "fca_stft",
                     "fca_istft", "fca_multi_init", "fca_multi_em_step", "fca_multi_separate", "fca_multi_timing"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def fca_last_error(ctx=None) -> str:
    h = ctx.handle if ctx is not None else None
    return lib().fca_last_error(h).decode()


def _check(status: int, ctx=None, allow=()):
    if status != FCA_OK and status not in allow:
        raise FcaError(status, fca_last_error(ctx))
    return status


def _stream_handle(device: torch.device):
    if device.type == "cuda":
        return torch.cuda.current_stream(device).cuda_stream
    return None


def _as_tensor(a, dtype=None):
    if a is None:
        return None
    t = torch.from_numpy(np.ascontiguousarray(a)) if isinstance(a, np.ndarray) else a
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return t


@dataclass
class Ctx:
    """Handle of an fca_ctx plus the shapes needed to size outputs."""
    handle: int
    Ms: list
    Ns: list
    F: int
    prec: int
    device: torch.device

    @property
    def B(self):
        return len(self.Ms)

    @property
    def real_dtype(self):
        return torch.float64 if self.prec == FCA_FP64 else torch.float32

    @property
    def complex_dtype(self):
        return torch.complex128 if self.prec == FCA_FP64 else torch.complex64


def _problem(y, R0, v0, prec, stream):
    """fca_problem for y[f, n, m] (any strides); keeps the tensors alive via the return."""
    cdt = torch.complex128 if prec == FCA_FP64 else torch.complex64
    rdt = torch.float64 if prec == FCA_FP64 else torch.float32
    y = _as_tensor(y, cdt)
    if y.dim() != 3:
        raise ValueError("y must be [F, N, M]")
    F, N, M = y.shape
    R0 = _as_tensor(R0, torch.complex128)
    v0 = _as_tensor(v0, rdt)
    if R0 is not None:
        R0 = R0.contiguous()
        if tuple(R0.shape) != (2, F, M, M):
            raise ValueError("R0 must be [2, F, M, M]")
    if v0 is not None:
        v0 = v0.contiguous()
        if tuple(v0.shape) != (2, F, N):
            raise ValueError("v0 must be [2, F, N]")
    p = fca_problem(M=M, F=F, N=N, prec=prec, y=y.data_ptr(), y_stride_f=y.stride(0),
                    y_stride_n=y.stride(1), y_stride_m=y.stride(2),
                    R0=R0.data_ptr() if R0 is not None else None,
                    v0=v0.data_ptr() if v0 is not None else None, stream=stream)
    return p, (y, R0, v0), (M, F, N)


def fca_init(y, R0=None, v0=None, prec=FCA_FP32_BULK) -> Ctx:
    """Create a context for one mixture y[f, n, m] (torch or numpy)."""
    return fca_init_batch([y], None if R0 is None else [R0], None if v0 is None else [v0], prec)


def fca_init_batch(ys, R0s=None, v0s=None, prec=FCA_FP32_BULK) -> Ctx:
    ys = [_as_tensor(y) for y in ys]
    device = ys[0].device if isinstance(ys[0], torch.Tensor) else torch.device("cpu")
    if device.type != "cuda":
        device = torch.device("cuda", torch.cuda.current_device())
    stream = _stream_handle(device)
    R0s = R0s or [None] * len(ys)
    v0s = v0s or [None] * len(ys)
    probs, keep, shapes = [], [], []
    for y, R0, v0 in zip(ys, R0s, v0s):
        p, k, s = _problem(y, R0, v0, prec, stream)
        probs.append(p)
        keep.append(k)
        shapes.append(s)
    arr = (fca_problem * len(probs))(*probs)
    h = ctypes.c_void_p()
    _check(lib().fca_init_batch(arr, len(probs), ctypes.byref(h)))
    del keep
    return Ctx(handle=h.value, Ms=[s[0] for s in shapes], Ns=[s[2] for s in shapes], F=shapes[0][1],
               prec=prec, device=device)


def fca_reset(ctx: Ctx):
    _check(lib().fca_reset(ctx.handle), ctx)


def fca_set_start(ctx: Ctx, b: int, R0=None, v0=None):
    """New initial values for mixture b (None = default R / plain powers);
    resets that mixture and makes it active. Tensors may be on host or device."""
    R0 = _as_tensor(R0, torch.complex128)
    v0 = _as_tensor(v0, ctx.real_dtype)
    M, N = ctx.Ms[b], ctx.Ns[b]
    if R0 is not None:
        R0 = R0.contiguous()
        if tuple(R0.shape) != (2, ctx.F, M, M):
            raise ValueError("R0 must be [2, F, M, M]")
    if v0 is not None:
        v0 = v0.contiguous()
        if tuple(v0.shape) != (2, ctx.F, N):
            raise ValueError("v0 must be [2, F, N]")
    _check(lib().fca_set_start(ctx.handle, b, R0.data_ptr() if R0 is not None else None,
                               v0.data_ptr() if v0 is not None else None), ctx)


def fca_set_active(ctx: Ctx, b: int, active: bool):
    """Include (True) or exclude (False) mixture b from later EM calls."""
    _check(lib().fca_set_active(ctx.handle, b, 1 if active else 0), ctx)


def fca_em_step(ctx: Ctx, iters: int, want_loglik=True, want_R=True, want_v=True, allow_flags=False,
                _entry="fca_em_step"):
    """Run `iters` EM iterations. Returns (loglik [B, max(iters,1)] float64,
    R list of [2, F, M, M] complex128, v list of [2, F, N]) on the context's
    device (entries not requested are None)."""
    B, F = ctx.B, ctx.F
    dev = ctx.device
    ll = torch.empty((B, max(iters, 1)), dtype=torch.float64, device=dev) if want_loglik else None
    nR = sum(2 * F * m * m for m in ctx.Ms)
    nv = sum(2 * F * n for n in ctx.Ns)
    R = torch.empty(nR, dtype=torch.complex128, device=dev) if want_R else None
    v = torch.empty(nv, dtype=ctx.real_dtype, device=dev) if want_v else None
    allow = (FCA_E_NOT_PD, FCA_E_NONFINITE) if allow_flags else ()
    _check(getattr(lib(), _entry)(ctx.handle, iters, ll.data_ptr() if ll is not None else None,
                             R.data_ptr() if R is not None else None,
                             v.data_ptr() if v is not None else None), ctx, allow)
    Rs = vs = None
    if want_R:
        Rs, o = [], 0
        for m in ctx.Ms:
            Rs.append(R[o:o + 2 * F * m * m].view(2, F, m, m))
            o += 2 * F * m * m
    if want_v:
        vs, o = [], 0
        for n in ctx.Ns:
            vs.append(v[o:o + 2 * F * n].view(2, F, n))
            o += 2 * F * n
    return ll, Rs, vs


def fca_conv_em_step(ctx: Ctx, iters: int, want_loglik=True, want_R=True, want_v=True, allow_flags=False):
    """As fca_em_step, computed by the conventional frame-wise EM kernel."""
    return fca_em_step(ctx, iters, want_loglik, want_R, want_v, allow_flags, _entry="fca_conv_em_step")


def fca_separate(ctx: Ctx):
    """MMSE source images, list of [2, F, N, M] complex tensors (one per mixture)."""
    tot = sum(2 * ctx.F * n * m for n, m in zip(ctx.Ns, ctx.Ms))
    x = torch.empty(tot, dtype=ctx.complex_dtype, device=ctx.device)
    _check(lib().fca_separate(ctx.handle, x.data_ptr()), ctx)
    out, o = [], 0
    for n, m in zip(ctx.Ns, ctx.Ms):
        out.append(x[o:o + 2 * ctx.F * n * m].view(2, ctx.F, n, m))
        o += 2 * ctx.F * n * m
    return out


def fca_status_per_freq(ctx: Ctx) -> np.ndarray:
    flags = np.zeros((ctx.B, ctx.F), np.int32)
    _check(lib().fca_status_per_freq(ctx.handle, flags.ctypes.data), ctx)
    return flags


def fca_loglik_per_freq(ctx: Ctx, rows: int = 1) -> torch.Tensor:
    """[rows, B, F] float64 device tensor: per-frequency log-likelihood of
    the last `rows` iterations of the previous EM call (NaN for mixtures that
    call skipped)."""
    out = torch.empty((rows, ctx.B, ctx.F), dtype=torch.float64, device=ctx.device)
    _check(lib().fca_loglik_per_freq(ctx.handle, int(rows), out.data_ptr()), ctx)
    return out


def fca_em_solve_noalloc(y: torch.Tensor, v: torch.Tensor, N: int, iters: int, use_v0: bool = False,
                         loglik=None, R_out=None, flags_out=None):
    """The allocation-free plain-start EM of one mixture: y device [F, M,
    pitch] complex (complex128: FP64, complex64: FP32 bulk) with N <= pitch
    frames per row, v device [2, F, pitch] real (in: v0 if use_v0; out: the
    powers after the iterations); loglik [max(iters, 1)] float64, R_out
    [2, F, M, M] complex128 and flags_out [F] int32 preallocated device
    tensors or None. Enqueued on the current stream."""
    F, M, pitch = y.shape
    prec = FCA_FP64 if y.dtype == torch.complex128 else FCA_FP32_BULK

    def ptr(t):
        return t.data_ptr() if t is not None else None
    _check(lib().fca_em_solve_noalloc(M, F, int(N), prec, y.data_ptr(), pitch, v.data_ptr(), int(use_v0),
                                      int(iters), ptr(loglik), ptr(R_out), ptr(flags_out),
                                      _stream_handle(y.device)))


def fca_stft_frames(T: int, L: int = 1024) -> int:
    return int(lib().fca_stft_frames(int(T), int(L)))


def fca_stft(x: torch.Tensor, L: int = 1024) -> torch.Tensor:
    """STFT of real device signals x [M, T] (float32: complex64 out, float64:
    complex128 out) -> X [F, N, M] (F = L/2 + 1), the EM's mixture layout."""
    M, T = x.shape
    x = x.contiguous()
    prec = FCA_FP64 if x.dtype == torch.float64 else FCA_FP32_BULK
    cdt = torch.complex128 if prec == FCA_FP64 else torch.complex64
    X = torch.empty((L // 2 + 1, fca_stft_frames(T, L), M), dtype=cdt, device=x.device)
    _check(lib().fca_stft(M, T, L, prec, x.data_ptr(), X.data_ptr(), _stream_handle(x.device)))
    return X


def fca_istft(X: torch.Tensor, T: int, L: int = 1024) -> torch.Tensor:
    """Overlap-add synthesis of device spectra X [F, N, M] -> x [M, T] real."""
    F, N, M = X.shape
    X = X.contiguous()
    prec = FCA_FP64 if X.dtype == torch.complex128 else FCA_FP32_BULK
    rdt = torch.float64 if prec == FCA_FP64 else torch.float32
    x = torch.empty((M, T), dtype=rdt, device=X.device)
    _check(lib().fca_istft(M, T, L, prec, X.data_ptr(), x.data_ptr(), _stream_handle(X.device)))
    return x


# ------------------------------------------------------------------ J sources
@dataclass
class MultiCtx:
    """Handle of an fca_mctx (one mixture, J sources) plus its shapes."""
    handle: int
    J: int
    M: int
    F: int
    N: int
    prec: int
    device: torch.device

    @property
    def real_dtype(self):
        return torch.float64 if self.prec == FCA_FP64 else torch.float32

    @property
    def complex_dtype(self):
        return torch.complex128 if self.prec == FCA_FP64 else torch.complex64


def _mcheck(status: int, ctx=None, allow=()):
    if status != FCA_OK and status not in allow:
        raise FcaError(status, fca_multi_last_error(ctx))
    return status


def fca_multi_init(y, J: int, R0=None, v0=None, prec=FCA_FP32_BULK) -> MultiCtx:
    """J-source context for one mixture y[f, n, m]; R0 [J, F, M, M]
    complex128 and v0 [J, F, N] (prec reals) optional, host or device."""
    y = _as_tensor(y)
    device = y.device if y.device.type == "cuda" else torch.device("cuda", torch.cuda.current_device())
    p, keep, (M, F, N) = _problem(y, None, None, prec, _stream_handle(device))
    R0 = _as_tensor(R0, torch.complex128)
    v0 = _as_tensor(v0, torch.float64 if prec == FCA_FP64 else torch.float32)
    if R0 is not None:
        R0 = R0.contiguous()
        if tuple(R0.shape) != (J, F, M, M):
            raise ValueError("R0 must be [J, F, M, M]")
    if v0 is not None:
        v0 = v0.contiguous()
        if tuple(v0.shape) != (J, F, N):
            raise ValueError("v0 must be [J, F, N]")
    h = ctypes.c_void_p()
    _mcheck(lib().fca_multi_init(ctypes.byref(p), J, R0.data_ptr() if R0 is not None else None,
                                 v0.data_ptr() if v0 is not None else None, ctypes.byref(h)))
    del keep
    return MultiCtx(handle=h.value, J=J, M=M, F=F, N=N, prec=prec, device=device)


def fca_multi_em_step(ctx: MultiCtx, iters: int, want_loglik=True, want_R=True, want_v=True, allow_flags=False):
    """Run `iters` iterations. Returns (loglik [max(iters, 1)] float64,
    R [J, F, M, M] complex128, v [J, F, N]) on the device (None if not asked)."""
    dev = ctx.device
    ll = torch.empty(max(iters, 1), dtype=torch.float64, device=dev) if want_loglik else None
    R = torch.empty((ctx.J, ctx.F, ctx.M, ctx.M), dtype=torch.complex128, device=dev) if want_R else None
    v = torch.empty((ctx.J, ctx.F, ctx.N), dtype=ctx.real_dtype, device=dev) if want_v else None
    allow = (FCA_E_NOT_PD, FCA_E_NONFINITE) if allow_flags else ()
    _mcheck(lib().fca_multi_em_step(ctx.handle, iters, ll.data_ptr() if ll is not None else None,
                                    R.data_ptr() if R is not None else None,
                                    v.data_ptr() if v is not None else None), ctx, allow)
    return ll, R, v


def fca_multi_separate(ctx: MultiCtx) -> torch.Tensor:
    """MMSE source images [J, F, N, M] complex (prec) on the device."""
    x = torch.empty((ctx.J, ctx.F, ctx.N, ctx.M), dtype=ctx.complex_dtype, device=ctx.device)
    _mcheck(lib().fca_multi_separate(ctx.handle, x.data_ptr()), ctx)
    return x


def fca_multi_timing(ctx: MultiCtx, enable: bool):
    """(ms, launches) of the iteration kernel since the previous call; enable
    switches event timing of later fca_multi_em_step calls on or off."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _mcheck(lib().fca_multi_timing(ctx.handle, 1 if enable else 0, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


def fca_multi_last_error(ctx: MultiCtx = None) -> str:
    return lib().fca_multi_last_error(ctx.handle if ctx is not None else None).decode()


def fca_multi_destroy(ctx: MultiCtx):
    if ctx is not None and ctx.handle:
        lib().fca_multi_destroy(ctx.handle)
        ctx.handle = None


def fca_destroy(ctx: Ctx):
    if ctx is not None and ctx.handle:
        lib().fca_destroy(ctx.handle)
        ctx.handle = None


def fca_gevd(S1: torch.Tensor, S2: torch.Tensor):
    """Batched FP64 GEVD of device tensors S1, S2 [count, M, M] complex128.
    Returns (P [count, M, M], lam [count, M], flags [count])."""
    if S1.dtype != torch.complex128 or S2.dtype != torch.complex128:
        raise TypeError("S1 and S2 must be complex128")
    S1 = S1.contiguous()
    S2 = S2.contiguous()
    count, M, _ = S1.shape
    P = torch.empty_like(S1)
    lam = torch.empty((count, M), dtype=torch.float64, device=S1.device)
    flags = torch.empty((count,), dtype=torch.int32, device=S1.device)
    _check(lib().fca_gevd(M, count, S1.data_ptr(), S2.data_ptr(), P.data_ptr(), lam.data_ptr(),
                          flags.data_ptr(), _stream_handle(S1.device)))
    return P, lam, flags


def fca_timing(ctx: Ctx, enable: bool):
    """(EM-kernel milliseconds, launches) since the last call; sets timing on/off."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().fca_timing(ctx.handle, 1 if enable else 0, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


class fca_launch_group(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("threads", ctypes.c_int32), ("frames_per_thread", ctypes.c_int32),
                ("problems", ctypes.c_int32), ("max_frames", ctypes.c_int32)]


def fca_launch_groups(ctx: Ctx) -> list:
    """Launch groups as dicts (M, threads, frames_per_thread, problems, max_frames)."""
    n = ctypes.c_int32()
    _check(lib().fca_launch_groups(ctx.handle, None, 0, ctypes.byref(n)), ctx)
    arr = (fca_launch_group * max(n.value, 1))()
    _check(lib().fca_launch_groups(ctx.handle, arr, n.value, ctypes.byref(n)), ctx)
    return [{k: getattr(arr[i], k) for k, _ in fca_launch_group._fields_} for i in range(n.value)]


def fca_set_launch_shape(ctx: Ctx, group: int, threads: int, streamed: bool = False):
    _check(lib().fca_set_launch_shape(ctx.handle, group, threads, 1 if streamed else 0), ctx)


def fca_autotune(ctx: Ctx, iters: int = 3):
    _check(lib().fca_autotune(ctx.handle, iters), ctx)


class Graph:
    """Device outputs of a captured step (loglik [B, max(iters,1)], flat R, v, x)."""

    def __init__(self, ctx: Ctx, iters: int, with_reset=True, want_loglik=True, want_R=True, want_v=True,
                 want_x=False):
        dev, F = ctx.device, ctx.F
        self.ctx = ctx
        self.loglik = torch.empty((ctx.B, max(iters, 1)), dtype=torch.float64, device=dev) if want_loglik else None
        self.R = (torch.empty(sum(2 * F * m * m for m in ctx.Ms), dtype=torch.complex128, device=dev)
                  if want_R else None)
        self.v = torch.empty(sum(2 * F * n for n in ctx.Ns), dtype=ctx.real_dtype, device=dev) if want_v else None
        self.x = (torch.empty(sum(2 * F * n * m for n, m in zip(ctx.Ns, ctx.Ms)), dtype=ctx.complex_dtype,
                              device=dev) if want_x else None)
        ptr = [t.data_ptr() if t is not None else None for t in (self.loglik, self.R, self.v, self.x)]
        _check(lib().fca_graph_capture(ctx.handle, iters, 1 if with_reset else 0, *ptr), ctx)

    def launch(self, count: int = 1, allow_flags=False):
        allow = (FCA_E_NOT_PD, FCA_E_NONFINITE) if allow_flags else ()
        _check(lib().fca_graph_launch(self.ctx.handle, count), self.ctx, allow)


def fca_graph_capture(ctx: Ctx, iters: int, with_reset=True, **want) -> Graph:
    """Capture one step (reset, iters EM iterations, outputs) into the context's graph."""
    return Graph(ctx, iters, with_reset, **want)


def fca_graph_launch(graph: Graph, count: int = 1, allow_flags=False):
    """Replay the captured step count times and wait."""
    graph.launch(count, allow_flags)


# ---------------------------------------------------------------------- learned initial powers (MLP)
class Mlp:
    """Handle of an fca_mlp (per-bin network predicting v1 / (v1 + v2))."""

    def __init__(self, M: int, seed: int = 0, max_batch: int = 8192, device=None, hidden: int = 256):
        self.device = torch.device(device or "cuda:0")
        self.M = M
        self.hidden = hidden
        self.max_batch = max_batch
        h = ctypes.c_void_p()
        self.stream = _stream_handle(self.device)
        st = lib().fca_mlp_create(M, hidden, seed, max_batch, self.stream, ctypes.byref(h))
        if st != FCA_OK:
            raise FcaError(st, lib().fca_mlp_last_error(None).decode())
        self.handle = h.value
        self.num_params = int(lib().fca_mlp_num_params(self.handle))

    def _check(self, st):
        if st != FCA_OK:
            raise FcaError(st, lib().fca_mlp_last_error(self.handle).decode())

    def close(self):
        if self.handle:
            lib().fca_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fca_mlp_create(M: int, seed: int = 0, max_batch: int = 8192, hidden: int = 256) -> Mlp:
    return Mlp(M, seed, max_batch, hidden=hidden)


def fca_mlp_destroy(m: Mlp):
    m.close()


def fca_mlp_num_params(m: Mlp) -> int:
    return m.num_params


def fca_mlp_last_error(m: Mlp = None) -> str:
    return lib().fca_mlp_last_error(m.handle if m is not None else None).decode()


def fca_mlp_get_params(m: Mlp) -> np.ndarray:
    out = np.zeros(m.num_params, np.float32)
    m._check(lib().fca_mlp_get_params(m.handle, out.ctypes.data))
    return out


def fca_mlp_set_params(m: Mlp, params: np.ndarray):
    params = np.ascontiguousarray(params, dtype=np.float32)
    assert params.shape == (m.num_params,)
    m._check(lib().fca_mlp_set_params(m.handle, params.ctypes.data))


def _dev(t, dtype):
    t = _as_tensor(t, dtype)
    return t.to("cuda").contiguous() if t.device.type != "cuda" else t.contiguous()


def fca_mlp_forward(m: Mlp, y, fpos) -> torch.Tensor:
    """r for bins y [n, M] complex64 with positions fpos [n] (device tensors or numpy)."""
    y = _dev(y, torch.complex64)
    fpos = _dev(fpos, torch.float32)
    n = y.shape[0]
    r = torch.empty(n, dtype=torch.float32, device=y.device)
    m._check(lib().fca_mlp_forward(m.handle, y.data_ptr(), fpos.data_ptr(), n, r.data_ptr()))
    return r


def fca_mlp_backward(m: Mlp, y, fpos, target, want_grads=False):
    """(loss, grads or None) of the mean binary cross-entropy on one batch."""
    y = _dev(y, torch.complex64)
    fpos = _dev(fpos, torch.float32)
    target = _dev(target, torch.float32)
    loss = ctypes.c_double()
    g = np.zeros(m.num_params, np.float32) if want_grads else None
    m._check(lib().fca_mlp_backward(m.handle, y.data_ptr(), fpos.data_ptr(), target.data_ptr(), y.shape[0],
                                    ctypes.byref(loss), g.ctypes.data if g is not None else None))
    return loss.value, g


def fca_mlp_adamw(m: Mlp, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4):
    m._check(lib().fca_mlp_adamw(m.handle, lr, beta1, beta2, eps, weight_decay))


def fca_mlp_init_powers(m: Mlp, y) -> torch.Tensor:
    """Learned start v0 [2, F, N] (float32, device) for y [F, N, M] complex64."""
    y = _dev(y, torch.complex64)
    F, N, M = y.shape
    v0 = torch.empty((2, F, N), dtype=torch.float32, device=y.device)
    m._check(lib().fca_mlp_init_powers(m.handle, y.data_ptr(), F, N, v0.data_ptr()))
    if torch.cuda.current_stream(y.device).cuda_stream != m.stream:
        torch.cuda.synchronize(y.device)  # the kernel ran on the network's stream
    return v0


def fca_mlp_init_powers_batch(m: Mlp, ys) -> list:
    """Learned starts of several mixtures (each y [F, N_b, M] complex64, one F)
    in one launch: list of v0 [2, F, N_b] float32 views of one device buffer."""
    ys = [_dev(y, torch.complex64) for y in ys]
    F, M = ys[0].shape[0], ys[0].shape[2]
    if any(y.shape[0] != F or y.shape[2] != M for y in ys):
        raise ValueError("fca_mlp_init_powers_batch: every mixture needs the same F and M")
    Ns = [int(y.shape[1]) for y in ys]
    buf = torch.empty(sum(2 * F * n for n in Ns), dtype=torch.float32, device=ys[0].device)
    v0s, o = [], 0
    for n in Ns:
        v0s.append(buf[o:o + 2 * F * n].view(2, F, n))
        o += 2 * F * n
    k = len(ys)
    yp = (ctypes.c_void_p * k)(*[y.data_ptr() for y in ys])
    vp_ = (ctypes.c_void_p * k)(*[v.data_ptr() for v in v0s])
    nn = (ctypes.c_int32 * k)(*Ns)
    m._check(lib().fca_mlp_init_powers_batch(m.handle, k, yp, F, nn, vp_))
    if torch.cuda.current_stream(ys[0].device).cuda_stream != m.stream:
        torch.cuda.synchronize(ys[0].device)
    return v0s


def fca_set_learned_starts(ctx: Ctx, m: Mlp, mixtures=None):
    """Learned starts from the mixtures the (FP32) context holds, for the
    listed mixtures (default: all), in one inference launch; each is reset
    to its new start and made active."""
    if mixtures is None:
        n, arr = ctx.B, None
    else:
        mixtures = [int(b) for b in mixtures]
        n, arr = len(mixtures), (ctypes.c_int32 * len(mixtures))(*mixtures)
    _check(lib().fca_set_learned_starts(ctx.handle, m.handle, n, arr), ctx)


def fca_set_mask_covariances(ctx: Ctx, mixtures=None, sharpen: float = 3.0, load: float = 1e-3):
    """Initial R_j from time-frequency masks made of the stored powers of the
    listed mixtures (default: all): r = v1 / (v1 + v2) sharpened to
    r^p / (r^p + (1 - r)^p), R_j = M A_j / tr A_j + load I with
    A_j = sum_n w_j y y^H (w_1 = r, w_2 = 1 - r); each mixture is reset to its
    new start and made active."""
    if mixtures is None:
        n, arr = ctx.B, None
    else:
        mixtures = [int(b) for b in mixtures]
        n, arr = len(mixtures), (ctypes.c_int32 * len(mixtures))(*mixtures)
    _check(lib().fca_set_mask_covariances(ctx.handle, n, arr, float(sharpen), float(load)), ctx)
