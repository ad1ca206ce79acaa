"""Benchmark of the FastFCA EM hot path on one MI355X.

Default workload: one synthetic array mixture, M = 4 microphones, F = 513
bins, N = 1000 frames, complex64 input, FP32 bulk arithmetic with FP64
eigendecomposition and log-likelihood sums, 50 EM iterations. One step is the
whole path on that input, with the input already resident in HBM: set the
initial values (plain start), 50 EM iterations returning the per-iteration
log-likelihood, R_j(f) and v_j(n,f), then the MMSE source images.

Metric: time-frequency-bin EM updates per second = F * N * iterations / step
time. Prints one JSON line with
  - a roofline entry for the EM-iteration kernel (timed with HIP events on
    the stream it runs on): algorithmic bytes (8 M + 16 per bin and
    iteration: y read, v read and written) over the launch time, against the
    8 TB/s HBM peak, with the flop view beside it;
  - the error of the GPU result against the CPU oracle (conventional FCA EM,
    FP64) on the frequencies whose true covariances have condition number
    <= 1e3, and by condition-number class on the others;
  - the conventional-EM kernel timed on the same workload (in-run baseline);
  - the same workload in the FP64 mode (time per step and its oracle error);
  - the CPU oracle's own throughput on the host's cores;
  - time to target (unless --no-ttt): held-out mixtures with AR(1) powers,
    plain FastFCA FP32 one mixture at a time against batched runs with and
    without the learned start (see time_to_target).

Other workloads (--workload): "batched" = 64 mixtures with N uniform in
[200, 2000] and M drawn from {2, 4, 8}; "large" = 16 mixtures, M = 8,
F = 1025, N = 8000, 100 iterations (frames streamed); "time-to-target" =
the time-to-target comparison alone; "ttt-tune" = the choice of the learned
path's settings (mask sharpening, start-comparison iteration, stop-check
chunks) on mixtures disjoint from the evaluation ones; "stft" = the STFT
analysis and synthesis of a four-microphone recording of 1024 s at the paper's
settings (samples/s, HBM roofline of both kernels); "multi" = the J-source
EM (J = 3 and 4) on one array mixture M = 4, F = 513, N = 1000.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TF-bin EM updates/sec at M=4; time-to-target log-lik vs plain FastFCA"
PEAK_HBM_GBS = 8000.0                # MI355X published HBM3E bandwidth
PEAK_FP32_VECTOR_TFLOPS = 157.3      # MI355X published FP32 vector peak (packed instructions)
FP32_UNPACKED_TFLOPS = 78.6          # the same without packed FP32, which every build here disables
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "em_kernel_array_m4_traffic.json")
# the EM kernel's own sources: a change there makes the stored traffic stale
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1805_06572_amd", "csrc", f)
                  for f in ("fca_em.h", "fca_em_nt256.hip", "fca_device.h")]
KAPPA_GATE = 1e3                     # float-bulk parity gate on cond(R_true)


def flop_per_update(M: int) -> int:
    """Algorithmic flops of one bin through one iteration: y~ = P^H y (8 M^2),
    the S~ accumulation (16 M^2), the scalar E/M-step and log-likelihood (~25 M)."""
    return 24 * M * M + 25 * M


def bytes_per_update(M: int) -> int:
    """y read (8 M B, complex64), v read and written (2 x 8 B)."""
    return 8 * M + 16


STFT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stft1024_traffic.json")
STFT_SOURCES = [os.path.join(ROOT, "paper_1805_06572_amd", "csrc", "fca_stft.hip")]


def kernel_source_hash(sources=None) -> str:
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def load_traffic(path=TRAFFIC_FILE, sources=None, key="bytes_per_launch"):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    scaled by a copy-kernel calibration), if taken on the current kernel
    sources."""
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash(sources):
        return None
    return t.get(key)


def oracle_threads() -> int:
    return min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16))


def cpu_baseline(mixtures, iters: int, freqs_per_mixture: int, frames: int | None = None):
    """Time the CPU oracle (conventional EM, FP64) on a bounded sample of the
    workload: the given mixtures, evenly spaced frequencies (frequencies are
    independent EM problems, so a subset is an exact sub-problem) and
    optionally the first `frames` frames."""
    import numpy as np
    import oracle

    cores = oracle_threads()
    total_t, updates, desc = 0.0, 0, []
    for y in mixtures:
        F, N, _ = y.shape
        idx = np.linspace(0, F - 1, min(freqs_per_mixture, F)).round().astype(int)
        y64 = np.ascontiguousarray(np.asarray(y, dtype=np.complex128)[idx, :frames])
        S0, v0 = oracle.default_init(y64)
        oracle.em(y64[:1, :8], S0[:, :1], v0[:, :1, :8], 1, threads=cores)   # load + warm
        t0 = time.perf_counter()
        oracle.em(y64, S0, v0, iters, threads=cores)
        total_t += time.perf_counter() - t0
        updates += y64.shape[0] * y64.shape[1] * iters
        desc.append(f"{len(idx)}/{F} frequencies x {y64.shape[1]} frames")
    return {"value": updates / total_t, "unit": "updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{'; '.join(desc[:2])}{' ...' if len(desc) > 2 else ''} ({len(mixtures)} mixture(s)), "
                      f"{iters} iterations of the conventional FCA EM in FP64 ({total_t:.2f} s wall)"}


class Runner:
    """One context with device buffers for the outputs and a timed step."""

    def __init__(self, fca, ys, iters, prec, v0s=None):
        import torch
        self.fca, self.iters = fca, iters
        self.ctx = fca.fca_init_batch(ys, v0s=v0s, prec=prec)
        c = self.ctx
        dev = c.device
        self.ll = torch.empty((c.B, max(iters, 1)), dtype=torch.float64, device=dev)
        self.R = torch.empty(sum(2 * c.F * m * m for m in c.Ms), dtype=torch.complex128, device=dev)
        self.v = torch.empty(sum(2 * c.F * n for n in c.Ns), dtype=c.real_dtype, device=dev)
        self.x = torch.empty(sum(2 * c.F * n * m for n, m in zip(c.Ns, c.Ms)), dtype=c.complex_dtype, device=dev)
        self.lib = fca.lib()
        self.ok = (fca.FCA_OK, fca.FCA_E_NOT_PD, fca.FCA_E_NONFINITE)

    def step(self, conventional=False, separate=True):
        fca, h = self.fca, self.ctx.handle
        st = self.lib.fca_reset(h)
        assert st == fca.FCA_OK, fca.fca_last_error(self.ctx)
        entry = self.lib.fca_conv_em_step if conventional else self.lib.fca_em_step
        st = entry(h, self.iters, self.ll.data_ptr(), self.R.data_ptr(), self.v.data_ptr())
        assert st in self.ok, fca.fca_last_error(self.ctx)
        if separate:
            st = self.lib.fca_separate(h, self.x.data_ptr())
            assert st == fca.FCA_OK, fca.fca_last_error(self.ctx)

    def timed(self, steps, warmup, **kw):
        """(ms per step, EM-kernel ms per step)."""
        import torch
        for _ in range(warmup):
            self.step(**kw)
        torch.cuda.synchronize()
        self.fca.fca_timing(self.ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step(**kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms, _ = self.fca.fca_timing(self.ctx, False)
        return dt * 1e3 / steps, ms / steps

    def graph_timed(self, steps, warmup, separate=True):
        """ms per step of the captured step (reset + iterations + LL, R, v
        out [+ separation]) replayed `steps` times back to back; the outputs
        land in the same buffers as step()."""
        import torch
        import ctypes
        x = self.x.data_ptr() if separate else None
        st = self.lib.fca_graph_capture(self.ctx.handle, self.iters, 1, self.ll.data_ptr(), self.R.data_ptr(),
                                        self.v.data_ptr(), ctypes.c_void_p(x) if x else None)
        assert st == self.fca.FCA_OK, self.fca.fca_last_error(self.ctx)
        if warmup:
            st = self.lib.fca_graph_launch(self.ctx.handle, warmup)
            assert st in self.ok, self.fca.fca_last_error(self.ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = self.lib.fca_graph_launch(self.ctx.handle, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert st in self.ok, self.fca.fca_last_error(self.ctx)
        return dt * 1e3 / steps

    def autotune(self, iters=3):
        self.fca.fca_autotune(self.ctx, iters)
        return [(g["M"], g["threads"], g["frames_per_thread"], g["problems"])
                for g in self.fca.fca_launch_groups(self.ctx)]

    def close(self):
        self.fca.fca_destroy(self.ctx)


def roofline_entry(kernel_ms, bytes_alg, flop, traffic, kernel_name):
    """The EM kernel against the HBM roofline: algorithmic bytes of one
    launch (all iterations of the call) over its duration; the flop view
    (24 M^2 + 25 M per bin and iteration) is kept beside it."""
    gbs = bytes_alg / (kernel_ms * 1e-3) / 1e9
    tflops = flop / (kernel_ms * 1e-3) / 1e12
    return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "traffic": traffic, "kernel": kernel_name, "kernel_ms_per_launch": kernel_ms,
            "algorithmic_bytes_per_launch": bytes_alg,
            "bytes_rule": "(8 M + 16) B per bin and iteration (y read, v read and written) x bins x iterations",
            "flop_view": {"flop_per_launch": flop, "achieved_tflops": tflops,
                          "frac_of_157_3_packed_peak": tflops / PEAK_FP32_VECTOR_TFLOPS,
                          "frac_of_78_6_unpacked": tflops / FP32_UNPACKED_TFLOPS}}


def base_record(args, value, ms_per_step, config, metric=METRIC, unit="updates/s"):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": config}


# ---------------------------------------------------------------------------- workloads
def invariants(fca, R, gll_f):
    """Run metrics of the method's invariants on the final parameters
    R [2, F, M, M] (device, complex128) and the per-frequency log-likelihood
    rows gll_f [iters, F]: the library's FP64 generalized eigendecomposition of
    (R1, R2) must give P^H R2 P = I and P^H R1 P = diag(lambda) (the Appendix
    theorem), and the EM log-likelihood never decreases (Section 2)."""
    import numpy as np
    import torch
    R1, R2 = R[0].contiguous(), R[1].contiguous()
    P, lam, flags = fca.fca_gevd(R1, R2)
    PH = P.conj().transpose(-1, -2).contiguous()
    eye = torch.eye(R1.shape[-1], dtype=torch.complex128, device=R1.device)
    r2 = (torch.matmul(torch.matmul(PH, R2), P) - eye).abs().amax(dim=(-2, -1)).cpu().numpy()
    d1 = torch.matmul(torch.matmul(PH, R1), P) - torch.diag_embed(lam.to(torch.complex128))
    r1 = (d1.abs().amax(dim=(-2, -1)) / lam.abs().amax(dim=-1)).cpu().numpy()
    # FP64 residuals grow with the conditioning of R2 (near-singular at the
    # lowest frequencies, where the diffuse field is almost rank one)
    w = np.linalg.eigvalsh(R2.cpu().numpy())
    cond = w[:, -1] / np.maximum(w[:, 0], 1e-300)
    dll = np.diff(gll_f, axis=0)
    drops = dll < -1e-6 * np.abs(gll_f[1:])
    q = lambda a: {"median": float(np.median(a)), "p99": float(np.quantile(a, 0.99)), "max": float(a.max())}
    return {"gevd_PH_R2_P_minus_I": q(r2), "gevd_PH_R1_P_minus_Lambda_rel": q(r1),
            "gevd_residual_over_cond_eps_max": float(np.max(np.maximum(r1, r2) / (cond * 2.2e-16))),
            "cond_R2": q(cond),
            "gevd_flagged": int((flags != 0).sum()),
            "loglik_decreases": {"count": int(drops.sum()), "of": int(dll.size),
                                 "rule": "LL(l+1) < LL(l) - 1e-6 |LL(l+1)| per frequency"}}


def oracle_error(kappa, oflags, gflags, S, v, ll, gR, gv, gll_f):
    """GPU against the oracle, per frequency: relative 2-norm errors of v_j
    and R_j, and of the log-likelihood of every iterate summed over the
    gated frequencies (cond(R_true) <= 1e3, not flagged by the oracle); the
    other frequencies by condition-number class."""
    import numpy as np

    def rel(a, b, axes):
        return np.sqrt((np.abs(a - b) ** 2).sum(axes)) / np.sqrt((np.abs(b) ** 2).sum(axes))
    ev = rel(gv.astype(np.float64), v, (-1,)).max(0)
    eR = rel(gR, S, (-2, -1)).max(0)
    gate = (kappa <= KAPPA_GATE) & (oflags == 0)
    iters = gll_f.shape[0]
    want = ll[:iters, gate].sum(1)
    e_ll = np.abs(gll_f[:, gate].sum(1) - want) / np.abs(ll[:iters, gate]).sum(1)
    classes = []
    edges = [KAPPA_GATE, 1e5, 1e7, 1e10, np.inf]
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (kappa > lo) & (kappa <= hi) & (oflags == 0) & (gflags == 0)
        if sel.any():
            classes.append({"kappa": [lo, None if np.isinf(hi) else hi], "frequencies": int(sel.sum()),
                            "v_rel_err_max": float(ev[sel].max()), "R_rel_err_max": float(eR[sel].max())})
    return {"gate": f"cond(R_true) <= {KAPPA_GATE:g} and not flagged by the oracle",
            "gated_frequencies": int(gate.sum()), "of": int(len(kappa)),
            "v_rel_err_max": float(ev[gate].max()), "R_rel_err_max": float(eR[gate].max()),
            "loglik_rel_err_max": float(e_ll.max()),
            "gpu_flags_in_gate": int((gflags[gate] != 0).sum()),
            "oracle_flagged": int((oflags != 0).sum()), "gpu_flagged": int((gflags != 0).sum()),
            "ungated_by_kappa": classes,
            "metric": "per frequency ||gpu - oracle|| / ||oracle|| (v over frames, R Frobenius), max over "
                      "frequencies and sources; loglik: |sum over gated f| error / sum of |terms|, max over "
                      "iterations"}


def run_array(args):
    import numpy as np
    import torch
    from paper_1805_06572_amd import fca, synth

    mx = synth.array_mixture(args.M, args.F, args.N, seed=1, complex64=True)
    y = torch.from_numpy(mx.y).cuda()
    torch.cuda.synchronize()
    if args.copy_calibration:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    L = args.iters
    run = Runner(fca, [y], L, fca.FCA_FP32_BULK)
    shapes = run.autotune() if args.autotune else None
    eager_ms, em_ms = run.timed(args.steps, args.warmup)
    ms_step = run.graph_timed(args.steps, args.warmup) if args.graph else eager_ms
    F, N, M = args.F, args.N, args.M
    # the outputs of the last timed step, before the conventional kernel reuses the buffers
    lls = run.ll.cpu().numpy()[0]
    gll_f = fca.fca_loglik_per_freq(run.ctx, L).cpu().numpy()[:, 0]
    inv = invariants(fca, run.R.view(2, F, M, M), gll_f)
    gR = run.R.view(2, F, M, M).cpu().numpy()
    gv = run.v.view(2, F, N).cpu().numpy()
    flags = fca.fca_status_per_freq(run.ctx)[0]
    conv_steps = max(1, args.steps // 10)
    _, conv_ms = run.timed(conv_steps, 1, conventional=True, separate=False)
    conv_flags = fca.fca_status_per_freq(run.ctx)[0]
    run.close()
    # the same workload in FP64 arithmetic throughout (the precise mode), eager steps
    run64 = Runner(fca, [y.to(torch.complex128)], L, fca.FCA_FP64)
    ms64, em64 = run64.timed(conv_steps, 1)
    gR64 = run64.R.view(2, F, M, M).cpu().numpy()
    gv64 = run64.v.view(2, F, N).cpu().numpy()
    gll64 = fca.fca_loglik_per_freq(run64.ctx, L).cpu().numpy()[:, 0]
    flags64 = fca.fca_status_per_freq(run64.ctx)[0]
    run64.close()

    updates = F * N * L
    rec = base_record(args, updates / (ms_step * 1e-3), ms_step,
                      {"workload": f"array mixture M={M} F={F} N={N}, {L} EM iterations, plain start",
                       "mixtures": 1, "M": M, "F": F, "N": N, "iterations": L,
                       "precision": "f32 per-bin arithmetic; f64 eigendecomposition and sums",
                       "step": "reset + em_step(loglik, R, v) + separate" +
                               (", captured in one HIP graph and replayed" if args.graph else ""),
                       "launch_shapes": shapes})
    rec["eager_ms_per_step"] = eager_ms
    rec["roofline"] = roofline_entry(em_ms, bytes_per_update(M) * updates, flop_per_update(M) * updates,
                                     load_traffic() if M == 4 else None,
                                     "em_kernel (one launch runs all iterations, one workgroup per frequency)")
    rec["in_run_baseline"] = {"kernel": "conv_em_kernel (conventional frame-wise EM, same workload)",
                              "kernel_ms_per_step": conv_ms, "updates_per_s": updates / (conv_ms * 1e-3),
                              "fastfca_kernel_speedup": conv_ms / em_ms,
                              "flagged_frequencies": int((conv_flags != 0).sum())}
    rec["fp64_variant"] = {"dtype": "f64", "ms_per_step": ms64, "updates_per_s": updates / (ms64 * 1e-3),
                           "em_kernel_ms_per_launch": em64, "flagged_frequencies": int((flags64 != 0).sum()),
                           "step": "reset + em_step(loglik, R, v) + separate, eager"}
    rec["loglik_first_last"] = [float(lls[0]), float(lls[-1])]
    rec["flagged_frequencies"] = int((flags != 0).sum())
    rec["invariants"] = inv
    if not args.no_cpu_baseline:
        # the oracle on every frequency and frame of the same input and start:
        # the CPU baseline and the error of the GPU result
        import oracle
        y64 = mx.y.astype(np.complex128)
        S0, v0 = oracle.default_init(y64)
        cores = oracle_threads()
        oracle.em(y64[:1, :8], S0[:, :1], v0[:, :1, :8], 1, threads=cores)   # load + warm
        t0 = time.perf_counter()
        S, v, ll, oflags = oracle.em(y64, S0, v0, L, threads=cores)
        cpu_s = time.perf_counter() - t0
        rec["oracle_error"] = oracle_error(synth.condition_numbers(mx.R), oflags, flags, S, v, ll, gR, gv, gll_f)
        rec["fp64_variant"]["oracle_error"] = oracle_error(synth.condition_numbers(mx.R), oflags, flags64, S, v, ll,
                                                           gR64, gv64, gll64)
        rec["cpu_baseline"] = {"value": updates / cpu_s, "unit": "updates/s", "cores": cores, "kind": "oracle",
                               "sample": f"{F}/{F} frequencies x {N} frames (1 mixture), {L} iterations of the "
                                         f"conventional FCA EM in FP64 ({cpu_s:.2f} s wall)"}
    if args.ttt:
        rec["time_to_target"] = time_to_target(args)
    return rec


def run_batched(args):
    import numpy as np
    import torch
    from paper_1805_06572_amd import fca, synth

    rng = np.random.default_rng(2)
    B, F, L = 64, 513, args.iters
    Ns = rng.integers(200, 2001, size=B)
    Ms = rng.choice([2, 4, 8], size=B)
    ys = [synth.array_mixture_device(int(Ms[b]), F, int(Ns[b]), seed=1000 + b)[0] for b in range(B)]
    torch.cuda.synchronize()
    run = Runner(fca, ys, L, fca.FCA_FP32_BULK)
    shapes = run.autotune() if args.autotune else None
    eager_ms, em_ms = run.timed(args.steps, args.warmup)
    ms_step = run.graph_timed(args.steps, args.warmup) if args.graph else eager_ms
    flags = fca.fca_status_per_freq(run.ctx)
    run.close()
    updates = int(F * Ns.sum() * L)
    flop = int(sum(flop_per_update(int(m)) * F * int(n) * L for m, n in zip(Ms, Ns)))
    bts = int(sum(bytes_per_update(int(m)) * F * int(n) * L for m, n in zip(Ms, Ns)))
    rec = base_record(args, updates / (ms_step * 1e-3), ms_step,
                      {"workload": f"{B} array mixtures, F={F}, N uniform in [200, 2000], M in {{2, 4, 8}}, "
                                   f"{L} EM iterations, plain start, one batched context",
                       "mixtures": B, "F": F, "N_total": int(Ns.sum()),
                       "M_counts": {str(m): int((Ms == m).sum()) for m in (2, 4, 8)},
                       "iterations": L, "precision": "f32 per-bin arithmetic; f64 eigendecomposition and sums",
                       "step": "reset + em_step(loglik, R, v) + separate" +
                               (", captured in one HIP graph and replayed" if args.graph else ""),
                       "launch_shapes": shapes})
    rec["eager_ms_per_step"] = eager_ms
    rec["roofline"] = roofline_entry(em_ms, bts, flop, None,
                                     "em_kernel / em_stream_kernel, one launch per (M, frames-per-thread) "
                                     "group, groups concurrent (time from the first launch to the last end)")
    rec["flagged_frequencies"] = int((flags != 0).sum())
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline([ys[i].cpu().numpy() for i in range(2)], L, 64)
    return rec


def run_large(args):
    import torch
    from paper_1805_06572_amd import fca, synth

    B, M, F, N, L = 16, 8, 1025, 8000, args.iters
    gen = [synth.array_mixture_device(M, F, N, seed=4000 + b) for b in range(B)]
    ys, R_true0 = [g[0] for g in gen], gen[0][2]
    del gen
    torch.cuda.synchronize()
    run = Runner(fca, ys, L, fca.FCA_FP32_BULK)
    learned = None
    if args.learned_large:
        # learned start per mixture (M=8 network of width 64), kept where the
        # EM rates it above the plain start at iteration 0
        from paper_1805_06572_amd import learned_init
        t0 = time.perf_counter()
        net, _ = learned_init.train(M=M, F=F, steps=args.train_steps, batch=8192, seed=0, hidden=64)
        train_s = time.perf_counter() - t0
        chosen, ll_p, ll_l, _ = learned_init.choose_starts(net, run.ctx, ys)
        v0_mix0 = fca.fca_mlp_init_powers(net, ys[0]) if chosen[0] else None
        net.close()
        learned = {"hidden": 64, "train_steps": args.train_steps, "train_s": train_s,
                   "learned_start_chosen": int(chosen.sum()),
                   "ll_gain_after_1_iteration_where_chosen": float((ll_l - ll_p)[chosen].sum())}
    ms_step, em_ms = run.timed(args.steps, args.warmup)
    flags = fca.fca_status_per_freq(run.ctx)
    run_R, run_v = run.R[: 2 * F * M * M].clone(), run.v[: 2 * F * N].clone()   # mixture 0
    # in-run baseline: the conventional frame-wise EM on the same batch and start (its frames are
    # streamed from memory every pass too), one step after one warm-up step
    _, conv_ms = run.timed(1, 1, conventional=True, separate=False)
    conv_flags = fca.fca_status_per_freq(run.ctx)
    run.close()
    updates = B * F * N * L
    rec = base_record(args, updates / (ms_step * 1e-3), ms_step,
                      {"workload": f"{B} array mixtures, M={M}, F={F}, N={N}, {L} EM iterations, "
                                   f"{'learned start with plain fallback' if learned else 'plain start'} "
                                   "(frames streamed from memory every pass)",
                       "mixtures": B, "M": M, "F": F, "N": N, "iterations": L,
                       "precision": "f32 per-bin arithmetic; f64 eigendecomposition and sums"})
    bts = bytes_per_update(M) * B * F * N * L   # streamed: y and v move every iteration
    rec["roofline"] = roofline_entry(em_ms, bts, flop_per_update(M) * updates, None,
                                     "em_stream_kernel (frames re-read every iteration)")
    rec["flagged_frequencies"] = int((flags != 0).sum())
    rec["in_run_baseline"] = {"kernel": "conv_stream_kernel (conventional frame-wise EM, same workload, frames "
                                        "streamed)",
                              "kernel_ms_per_step": conv_ms, "updates_per_s": updates / (conv_ms * 1e-3),
                              "fastfca_kernel_speedup": conv_ms / em_ms,
                              "flagged_frequencies": int((conv_flags != 0).sum())}
    if learned:
        rec["learned_start"] = learned
    if args.no_cpu_baseline:
        return rec
    # error against the FP64 oracle on a subsample: mixture 0, 8 evenly spaced
    # frequencies (each frequency is an independent EM problem), same start and
    # iteration count; the oracle run is also the CPU baseline
    import numpy as np
    import oracle
    idx = np.linspace(0, F - 1, 8).round().astype(int)
    y64 = np.ascontiguousarray(ys[0].cpu().numpy().astype(np.complex128)[idx])
    S0, v0 = oracle.default_init(y64)
    if learned and v0_mix0 is not None:
        v0 = np.ascontiguousarray(v0_mix0.cpu().numpy().astype(np.float64)[:, idx])
    cores = oracle_threads()
    t0 = time.perf_counter()
    S, v, ll, oflags = oracle.em(y64, S0, v0, L, threads=cores)
    cpu_s = time.perf_counter() - t0
    gR = run_R[: 2 * F * M * M].view(2, F, M, M)[:, idx].cpu().numpy()
    gv = run_v[: 2 * F * N].view(2, F, N)[:, idx].cpu().numpy().astype(np.float64)

    def rel(a, b, axes):
        return np.sqrt((np.abs(a - b) ** 2).sum(axes)) / np.sqrt((np.abs(b) ** 2).sum(axes))
    ev, eR = rel(gv, v, (-1,)).max(0), rel(gR, S, (-2, -1)).max(0)
    kappa = synth.condition_numbers(R_true0[:, idx])
    good = kappa <= 1e3
    rec["oracle_error_subsample"] = {
        "sample": f"mixture 0, frequencies {idx.tolist()}, all {N} frames, {L} iterations, same start "
                  f"({'learned' if learned and v0_mix0 is not None else 'plain'})",
        "kappa_R_true": [float(k) for k in kappa],
        "v_rel_err": [float(e) for e in ev], "R_rel_err": [float(e) for e in eR],
        "v_rel_err_max_kappa_le_1e3": float(ev[good].max()) if good.any() else None,
        "R_rel_err_max_kappa_le_1e3": float(eR[good].max()) if good.any() else None,
        "oracle_flagged": int((oflags != 0).sum()), "gpu_flagged": int((flags[0, idx] != 0).sum())}
    rec["cpu_baseline"] = {"value": len(idx) * N * L / cpu_s, "unit": "updates/s", "cores": cores,
                           "kind": "oracle",
                           "sample": f"{len(idx)}/{F} frequencies x {N} frames of 1 mixture, {L} iterations "
                                     f"of the conventional FCA EM in FP64 ({cpu_s:.2f} s wall)"}
    return rec


def progress(msg: str):
    """One line on stderr when a phase of a long run ends (the JSON result
    line stays alone on stdout)."""
    print(msg, file=sys.stderr, flush=True)


def time_to_target(args, seed0: int = 3000, K: int | None = None, settings=None, widths=None):
    """Time to a target log-likelihood, on K held-out array mixtures (M = 4,
    F = 513, N = 1000, AR(1) log-powers, seeds seed0 .. seed0 + K - 1).

    Only frequencies whose true covariances have cond(R_true) <= 1e3 count
    (the trust mask; below that the array model is numerically singular and
    its log-likelihood untrusted). Target of a mixture: the masked sum of the
    log-likelihood that plain FastFCA (plain start, FP32 bulk, one mixture at
    a time) reaches after 50 iterations; reached at LL >= target - 1e-3 (target
    - LL(theta^0)). Paths:
      - plain FastFCA FP32 one mixture at a time (its time prorated to the
        iteration that reaches the target: step time x iterations / 50);
      - all mixtures in one batched context, plain start, each stopped once
        it reaches its target (or has converged);
      - the same with the learned start (network of each hidden width,
        trained on the device first, its training time reported apart) and
        the mask-based R, the plain start kept per mixture where it has the
        higher log-likelihood (fallback); wall time from the context holding
        the mixtures to the last one stopped, the network inference, masks,
        start comparison included.
    settings: (mask sharpening, start-comparison iteration, stop-check chunks)
    of the learned path."""
    import numpy as np
    import torch
    from paper_1805_06572_amd import fca, learned_init, schedule, synth

    M, F, N, L = 4, 513, 1000, 50
    K = args.mixtures if K is None else K
    sharpen, choice_iter, chunks_learned = settings or (args.mask_sharpen, args.choice_iter,
                                                        tuple(int(c) for c in args.chunks.split(",")))
    widths = widths or [int(h) for h in args.hidden.split(",")]
    gens = [synth.array_mixture_device(M, F, N, seed=seed0 + k, ar1=True) for k in range(K)]
    ys = [g[0] for g in gens]
    trust = np.stack([synth.condition_numbers(g[2]) <= KAPPA_GATE for g in gens])
    del gens
    w = torch.from_numpy(trust.astype(np.float64)).cuda()
    torch.cuda.synchronize()

    def masked(rows, k):   # [r, F] per-frequency values of mixture k -> [r]
        return torch.where(w[k] > 0, rows * w[k], torch.zeros_like(rows)).sum(-1)

    plain = []
    for k, y in enumerate(ys):
        run = Runner(fca, [y], L, fca.FCA_FP32_BULK)
        step_ms, _ = run.timed(1, 1, separate=False)
        rows = fca.fca_loglik_per_freq(run.ctx, L)[:, 0]
        fca.fca_em_step(run.ctx, 0, want_R=False, want_v=False, allow_flags=True)
        last = fca.fca_loglik_per_freq(run.ctx, 1)[:, 0]
        plain.append((step_ms, masked(torch.cat([rows, last]), k).cpu().numpy()))
        run.close()
    target = np.array([h[-1] for _, h in plain])
    thr = target - 1e-3 * (target - np.array([h[0] for _, h in plain]))

    def first_hit(h, t):
        hit = np.nonzero(np.asarray(h) >= t)[0]
        return int(hit[0]) if len(hit) else None

    plain_its = [first_hit(h, thr[k]) for k, (_, h) in enumerate(plain)]
    plain_ms = sum(ms * (L if it is None else it) / L for (ms, _), it in zip(plain, plain_its))
    progress(f"time to target: plain FP32 one mixture at a time, {plain_ms:.1f} ms")
    hit_rule, conv_rule = schedule.reached(thr), schedule.converged(1e-6)

    def stop(b, ll):
        return hit_rule(b, ll) or conv_rule(b, ll)

    def batched(net):
        """(wall ms, start ms, iterations run, iterations to target, learned kept)
        of the second of two identical runs (the first warms up)."""
        for _ in range(2):
            ctx = fca.fca_init_batch(ys, prec=fca.FCA_FP32_BULK)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            chosen, adv = np.zeros(K, dtype=bool), np.zeros(K, dtype=int)
            if net is not None:
                chosen, _, _, adv = learned_init.choose_starts(net, ctx, ys, choice_iter=choice_iter,
                                                               mask_sharpen=sharpen if sharpen > 0 else None)
            t2 = time.perf_counter()
            iters, hist = schedule.run_batch(ctx, 2 * L, chunks_learned if net is not None else (16, 8, 4),
                                             stop, weights=w)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            fca.fca_destroy(ctx)
        hits = [first_hit(h, thr[k]) for k, h in enumerate(hist)]
        hits = [None if h is None else int(h + a) for h, a in zip(hits, adv)]
        return (t3 - t1) * 1e3, (t2 - t1) * 1e3, np.asarray(iters) + adv, hits, chosen

    def stats(its):
        got = [i for i in its if i is not None]
        return {"mean": float(np.mean(got)) if got else None, "median": float(np.median(got)) if got else None,
                "reached": len(got), "of": len(its)}

    bp_ms, _, bp_run, bp_hits, _ = batched(None)
    progress(f"time to target: batched plain start, {bp_ms:.1f} ms")
    learned = []
    for H in widths:
        t0 = time.perf_counter()
        net, _ = learned_init.train(M=M, F=F, steps=args.train_steps, batch=8192, seed=0, hidden=H)
        train_s = time.perf_counter() - t0
        progress(f"time to target: width {H} trained in {train_s:.1f} s")
        bce, bce_const = learned_init.evaluate(net, n=65536, M=M, F=F)
        ms, start_ms, run_its, hits, chosen = batched(net)
        net.close()
        progress(f"time to target: width {H} learned start, {ms:.1f} ms")
        learned.append({"hidden": H, "ms": ms, "start_ms": start_ms,
                        "speedup_vs_plain_fp32_one_at_a_time": plain_ms / ms,
                        "speedup_vs_batched_plain": bp_ms / ms,
                        "iterations_to_target": stats(hits), "mean_iterations_run": float(np.mean(run_its)),
                        "learned_start_kept": int(np.sum(chosen)), "plain_fallbacks": int(K - np.sum(chosen)),
                        "train_s": train_s, "train_steps": args.train_steps, "heldout_bce": bce,
                        "constant_predictor_bce": bce_const})
    return {"mixtures": K, "seeds": [seed0, seed0 + K - 1], "M": M, "F": F, "N": N,
            "trusted_frequencies_mean": float(trust.sum(1).mean()),
            "target": "masked LL of plain FastFCA (FP32, plain start, one mixture at a time) after 50 "
                      "iterations; reached at target - 1e-3 (target - LL(theta^0)); mask cond(R_true) <= 1e3",
            "plain_fp32_one_at_a_time_ms": plain_ms,
            "plain_fp32_one_at_a_time_full_50_ms": float(sum(ms for ms, _ in plain)),
            "plain_iterations_to_target": stats(plain_its),
            "batched_plain_ms": bp_ms, "batched_plain_iterations_to_target": stats(bp_hits),
            "batched_plain_mean_iterations_run": float(np.mean(bp_run)),
            "learned": learned,
            "primary": {"hidden": learned[0]["hidden"], "ms": learned[0]["ms"],
                        "speedup_vs_plain_fp32_one_at_a_time": learned[0]["speedup_vs_plain_fp32_one_at_a_time"],
                        "speedup_vs_batched_plain": learned[0]["speedup_vs_batched_plain"]},
            "settings": {"mask_sharpen": sharpen, "mask_load": 1e-3, "start_comparison_iteration": choice_iter,
                         "stop_check_chunks": list(chunks_learned),
                         "chosen_on": "held-out seeds 5000.. (the ttt-tune workload), not on these mixtures"},
            "stop_rule": "reached target or masked LL rise below 1e-6 of the total, checked after each chunk"}


def run_time_to_target(args):
    out = time_to_target(args)
    head = out["learned"][0]
    rec = base_record(args, out["mixtures"] * out["F"] * out["N"] * head["mean_iterations_run"] / (head["ms"] * 1e-3),
                      head["ms"],
                      {"workload": f"time to target: {out['mixtures']} held-out array mixtures (AR(1) log-powers), "
                                   f"M=4, F=513, N=1000, learned start of hidden width {head['hidden']}",
                       "mixtures": out["mixtures"], "M": 4, "F": 513, "N": 1000, "hidden": head["hidden"]})
    rec["steps"], rec["warmup"] = 1, 1
    rec["time_to_target"] = out
    return rec


def hbm_entry(ms, nbytes, kernel, rule):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "traffic": None, "kernel": kernel, "kernel_ms_per_launch": ms, "algorithmic_bytes_per_launch": nbytes,
            "bytes_rule": rule}


def event_ms(fn, reps):
    """Mean duration of fn() over reps calls, HIP events on the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def run_stft(args):
    """The STFT front and back end at the paper's analysis settings (16 kHz,
    frames of 1024 samples, shift 512, square-root Hann window) on one
    4-microphone recording of 1024 s (the [F, N, 4] layout the EM takes),
    one call each way; the reconstruction error, and (the CPU baseline leg)
    the oracle's analysis of the first 4 s of channel 0, timed, with the
    GPU's error against it."""
    import numpy as np
    import torch
    from paper_1805_06572_amd import fca
    C, T, L = 4, 1024 * 16000, 1024
    g = torch.Generator(device="cuda").manual_seed(11)
    x = torch.randn((C, T), generator=g, device="cuda", dtype=torch.float32)
    X = fca.fca_stft(x, L)
    F, N, _ = X.shape
    ms_a = event_ms(lambda: fca.fca_stft(x, L), args.steps)
    ms_s = event_ms(lambda: fca.fca_istft(X, T, L), args.steps)
    xr = fca.fca_istft(X, T, L)
    rec_err = float((xr - x).abs().max() / x.abs().max())
    samples = C * T
    b_a = 4 * C * T + 8 * F * N * C
    rec = base_record(args, samples / (ms_a * 1e-3), ms_a + ms_s,
                      {"workload": f"STFT analysis and overlap-add synthesis, {C} channels x {T} samples "
                                   f"(a 4-microphone recording of 1024 s at 16 kHz), L = {L}, shift {L // 2}",
                       "channels": C, "samples_per_channel": T, "frame": L, "frames": N, "bins": F},
                      metric="STFT samples/s (analysis)", unit="samples/s")
    rec["synthesis_samples_per_s"] = samples / (ms_s * 1e-3)
    rec["roofline"] = hbm_entry(ms_a, b_a, "stft1024_kernel (16 transforms per workgroup)",
                                "4 B per input sample read once + 8 B per output bin written")
    rec["roofline"]["traffic"] = load_traffic(STFT_TRAFFIC_FILE, STFT_SOURCES, "stft1024_bytes_per_launch")
    rec["roofline_synthesis"] = hbm_entry(ms_s, b_a, "istft1024_kernel (16 transforms per workgroup)",
                                          "8 B per input bin read once + 4 B per output sample written")
    rec["roofline_synthesis"]["traffic"] = load_traffic(STFT_TRAFFIC_FILE, STFT_SOURCES, "istft1024_bytes_per_launch")
    rec["reconstruction_rel_err_max"] = rec_err
    if not args.no_cpu_baseline:
        import oracle.stft as ostft
        Th = 4 * 16000
        head = x[:1, :Th].double().cpu().numpy()
        t0 = time.perf_counter()
        want = ostft.stft(head, L)                   # [F, 126, 1]
        cpu_s = time.perf_counter() - t0
        full = (Th - 1) // (L // 2) - 1              # frames lying wholly in the first 4 s
        got = X[:, :full, :1].to(torch.complex128).cpu().numpy()
        err = float(np.max(np.abs(got - want[:, :full])) / np.max(np.abs(want[:, :full])))
        rec["oracle_error"] = {"sample": f"channel 0, frames 0..{full - 1} (the first 4 s)", "rel_err_max": err}
        rec["cpu_baseline"] = {"value": Th / cpu_s, "unit": "samples/s", "cores": 1, "kind": "oracle",
                               "sample": f"analysis of channel 0's first 4 s ({Th} samples) by the FP64 oracle "
                                         f"(defining DFT sum, {cpu_s:.2f} s wall)"}
    return rec


def multi_mixture(J, M, F, N, seed):
    """J far-field sources on the 4-microphone array: R_j(f) = a_j a_j^H +
    0.1 diffuse coherence (direction theta_j uniform in (0, pi)), v_j(n, f)
    Gamma(0.5, 1), images drawn as sqrt(v) R^(1/2) z."""
    import numpy as np
    from paper_1805_06572_amd import synth
    rng = np.random.default_rng(seed)
    G = synth.diffuse_coherence(M, F)
    y = np.zeros((F, N, M), np.complex128)
    for j in range(J):
        a = synth.steering_vectors(float(rng.uniform(0.0, np.pi)), M, F)
        R = a[:, :, None] * np.conj(a[:, None, :]) + 0.1 * G
        v = rng.gamma(0.5, 1.0, size=(F, N))
        y += synth.draw_images(R[None], v[None], synth.cn(rng, (1, F, N, M)), "eig")[0]
    return y


CHECK_ITERS = 5


def run_multi(args):
    """The J-source EM (approximate joint diagonalisation) on one array-style
    mixture of J sources, M = 4, F = 513, N = 1000, float bulk, `iters`
    iterations per call, for J = 3 and 4; in the CPU baseline leg the FP64
    oracle (oracle/multi.py) runs a few iterations on four frequencies,
    timed, and gives the GPU's error."""
    import numpy as np
    import torch
    from paper_1805_06572_amd import fca
    M, F, N, L = 4, 513, 1000, args.iters
    out = {}
    for J in (3, 4):
        y = multi_mixture(J, M, F, N, 40 + J)
        yd = torch.from_numpy(y.astype(np.complex64)).cuda()
        ctx = fca.fca_multi_init(yd, J, prec=fca.FCA_FP32_BULK)
        try:
            fca.fca_multi_em_step(ctx, 1, want_loglik=False, want_R=False, want_v=False, allow_flags=True)
            ms, kms = [], []
            for _ in range(args.steps):
                ctx2 = fca.fca_multi_init(yd, J, prec=fca.FCA_FP32_BULK)
                fca.fca_multi_timing(ctx2, True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ll, R_out, v_out = fca.fca_multi_em_step(ctx2, L, want_R=False, allow_flags=True)
                ms.append((time.perf_counter() - t0) * 1e3)
                k_ms, n_launch = fca.fca_multi_timing(ctx2, False)
                kms.append(k_ms / n_launch)
                if _ < args.steps - 1:
                    fca.fca_multi_destroy(ctx2)
            gll = ll.cpu().numpy()
            fca.fca_multi_destroy(ctx2)
            # a few iterations for the comparison with the oracle on four frequencies
            ctx2 = fca.fca_multi_init(yd, J, prec=fca.FCA_FP32_BULK)
            _, _, v_few = fca.fca_multi_em_step(ctx2, CHECK_ITERS, want_R=False, allow_flags=True)
            gv = v_few.double().cpu().numpy()
            fca.fca_multi_destroy(ctx2)
        finally:
            fca.fca_multi_destroy(ctx)
        t, tk = float(np.median(ms)), float(np.median(kms))
        bts = (8 * M + 8 * J) * F * N * L
        out[f"J{J}"] = {"ms_per_call": t, "updates_per_s": F * N * L / (t * 1e-3), "kernel_ms_per_launch": tk,
                        "roofline": hbm_entry(tk, bts, "em_multi_kernel (one workgroup per frequency, all iterations; "
                                              "HIP events on the context's stream)",
                                              "(8 M + 8 J) B per bin and iteration (y read, J powers read and written)"),
                        "loglik_first_last": [float(gll[0]), float(gll[-1])]}
        if not args.no_cpu_baseline:
            from oracle import multi
            idx = np.array([F // 8, 3 * F // 8, 5 * F // 8, 7 * F // 8])
            yc = y.astype(np.complex64).astype(np.complex128)[idx]
            t0 = time.perf_counter()
            S0, v0 = multi.default_start(yc, J)
            _, vo, _, _, _ = multi.fast_em(yc, S0, v0, CHECK_ITERS)
            cpu_s = time.perf_counter() - t0
            ev = float(np.max(np.sqrt((np.abs(gv[:, idx] - vo) ** 2).sum(-1)) / np.sqrt((np.abs(vo) ** 2).sum(-1))))
            out[f"J{J}"]["oracle_error"] = {"sample": f"v after {CHECK_ITERS} iterations, bins "
                                                      f"{', '.join(str(int(i)) for i in idx)}", "rel_err_max": ev}
            out[f"J{J}"]["cpu_baseline"] = {"value": len(idx) * N * CHECK_ITERS / cpu_s, "unit": "updates/s",
                                            "cores": 1, "kind": "oracle",
                                            "sample": f"{len(idx)}/{F} frequencies x {N} frames, {CHECK_ITERS} "
                                                      f"iterations of the FP64 AJD method ({cpu_s:.2f} s wall)"}
    rec = base_record(args, out["J3"]["updates_per_s"], out["J3"]["ms_per_call"],
                      {"workload": f"J-source EM, one mixture M={M} F={F} N={N}, {L} iterations, float bulk, "
                                   "plain start (J = 3 headline, J = 4 beside it)", "M": M, "F": F, "N": N,
                       "iterations": L},
                      metric="TF-bin EM updates/sec, J sources (approximate joint diagonalisation)")
    rec["roofline"] = out["J3"]["roofline"]
    if "cpu_baseline" in out["J3"]:
        rec["cpu_baseline"] = out["J3"]["cpu_baseline"]
    rec["per_J"] = out
    return rec


def run_ttt_tune(args):
    """Settings of the learned path (mask sharpening, start-comparison
    iteration, stop-check chunks) by wall time to target on 64 mixtures of
    seeds 5000.., disjoint from the evaluation mixtures."""
    grid = []
    for sharpen in (1.0, 2.0, 3.0, 4.0):
        for chunks in ((16, 4), (12, 4), (16, 8, 4), (8, 4)):
            grid.append((sharpen, 0, chunks))
    grid += [(3.0, 1, (16, 4)), (0.0, 1, (16, 8, 4))]
    res = []
    for st in grid:
        out = time_to_target(args, seed0=5000, K=64, settings=st, widths=[int(args.hidden.split(",")[0])])
        h = out["learned"][0]
        res.append({"mask_sharpen": st[0], "start_comparison_iteration": st[1], "chunks": list(st[2]),
                    "ms": h["ms"], "iterations_to_target": h["iterations_to_target"]["mean"],
                    "iterations_run": h["mean_iterations_run"], "batched_plain_ms": out["batched_plain_ms"]})
        print(json.dumps(res[-1]), file=sys.stderr, flush=True)
    best = min(res, key=lambda r: r["ms"])
    rec = base_record(args, None, best["ms"], {"workload": "ttt-tune: 64 array mixtures (AR(1)), seeds 5000..5063"})
    rec["grid"], rec["best"] = res, best
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="array",
                    choices=["array", "batched", "large", "time-to-target", "ttt-tune", "stft", "multi"])
    ap.add_argument("--no-ttt", dest="ttt", action="store_false",
                    help="array workload: skip the time-to-target comparison")
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--M", type=int, default=4)
    ap.add_argument("--F", type=int, default=513)
    ap.add_argument("--N", type=int, default=1000)
    ap.add_argument("--mixtures", type=int, default=256, help="time-to-target: held-out mixtures")
    ap.add_argument("--train-steps", type=int, default=None,
                    help="training steps of 8192 bins for the learned start (default: 20000 for "
                         "time-to-target, 2000 for the large workload)")
    ap.add_argument("--plain-large", dest="learned_large", action="store_false",
                    help="large workload: plain start only (no learned start)")
    ap.add_argument("--hidden", default="256,32",
                    help="time-to-target: hidden widths of the learned-start networks (the first one is the "
                         "primary figure)")
    ap.add_argument("--choice-iter", type=int, default=0,
                    help="time-to-target: EM iterations after which the plain and learned starts are compared")
    ap.add_argument("--mask-sharpen", type=float, default=3.0,
                    help="time-to-target: sharpening exponent of the masks that give the learned start its R "
                         "(0: plain R)")
    ap.add_argument("--chunks", default="16,4",
                    help="time-to-target: iterations per EM call of the learned path between stop checks (the "
                         "last one repeats)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="time the eager calls instead of the captured step")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device-to-device copy (3 times) so that "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE can be scaled to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the (mixture, frequency) "
              "problems shard with no per-iteration communication, but no multi-GPU path is "
              "implemented.", file=sys.stderr)
        sys.exit(2)
    if args.iters is None:
        args.iters = 100 if args.workload == "large" else 50
    if args.train_steps is None:
        args.train_steps = 2000 if args.workload == "large" else 20000
    import torch
    torch.cuda.set_device(0)
    runner = {"array": run_array, "batched": run_batched, "large": run_large,
              "time-to-target": run_time_to_target, "ttt-tune": run_ttt_tune, "stft": run_stft,
              "multi": run_multi}[args.workload]
    print(json.dumps(runner(args)), flush=True)


if __name__ == "__main__":
    main()
