"""Benchmark of the FastFCA EM hot path on one MI355X.

Default workload: one synthetic array mixture, M = 4 microphones, F = 513
bins, N = 1000 frames, complex64 input, FP32 bulk arithmetic with FP64
eigendecomposition and log-likelihood sums, 50 EM iterations. One step is the
whole path on that input, with the input already resident in HBM: set the
initial values (plain start), 50 EM iterations returning the per-iteration
log-likelihood, R_j(f) and v_j(n,f), then the MMSE source images.

Metric: time-frequency-bin EM updates per second = F * N * iterations / step
time. Prints one JSON line with a roofline entry for the EM-iteration kernel
(timed with HIP events on the stream it runs on), the conventional-EM kernel
timed on the same workload (in-run baseline) and the CPU oracle
(conventional FCA EM, FP64) on the host's cores.

Other workloads (--workload): "batched" = 64 mixtures with N uniform in
[200, 2000] and M drawn from {2, 4, 8}; "large" = 16 mixtures, M = 8,
F = 1025, N = 8000, 100 iterations (frames streamed); "time-to-target" =
learned start + one batched run of held-out mixtures against the plain start
run one mixture at a time.
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
PEAK_FP32_VECTOR_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "em_kernel_array_m4_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1805_06572_amd", "csrc", f)
                  for f in ("fca_em.h", "fca_em_nt256.hip", "fca_device.h", "fca_internal.h")]


def flop_per_update(M: int) -> int:
    """Algorithmic flops of one bin through one iteration: y~ = P^H y (8 M^2),
    the S~ accumulation (16 M^2), the scalar E/M-step and log-likelihood (~25 M)."""
    return 24 * M * M + 25 * M


def bytes_per_update(M: int) -> int:
    """y read (8 M B, complex64), v read and written (2 x 8 B)."""
    return 8 * M + 16


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def load_traffic():
    """Measured HBM bytes per EM launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    scaled by a copy-kernel calibration), if taken on the current kernel."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(mixtures, iters: int, freqs_per_mixture: int, frames: int | None = None):
    """Time the CPU oracle (conventional EM, FP64) on a bounded sample of the
    workload: the given mixtures, evenly spaced frequencies (frequencies are
    independent EM problems, so a subset is an exact sub-problem) and
    optionally the first `frames` frames."""
    import numpy as np
    import oracle

    cores = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
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


def roofline_entry(kernel_ms, flop, bytes_alg, traffic, kernel_name):
    achieved = flop / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic, "kernel": kernel_name,
            "kernel_ms_per_step": kernel_ms, "flop_per_step": flop, "algorithmic_bytes_per_step": bytes_alg,
            "hbm_equivalent_GBps": bytes_alg / (kernel_ms * 1e-3) / 1e9}


def base_record(args, value, ms_per_step, config):
    return {"metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": config}


# ---------------------------------------------------------------------------- workloads
def run_array(args):
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
    lls = run.ll.cpu().numpy()[0]
    flags = fca.fca_status_per_freq(run.ctx)[0]
    conv_steps = max(1, args.steps // 10)
    _, conv_ms = run.timed(conv_steps, 1, conventional=True, separate=False)
    conv_flags = fca.fca_status_per_freq(run.ctx)[0]
    run.close()

    F, N, M = args.F, args.N, args.M
    updates = F * N * L
    rec = base_record(args, updates / (ms_step * 1e-3), ms_step,
                      {"workload": f"array mixture M={M} F={F} N={N}, {L} EM iterations, plain start",
                       "mixtures": 1, "M": M, "F": F, "N": N, "iterations": L,
                       "precision": "f32 per-bin arithmetic; f64 eigendecomposition and sums",
                       "step": "reset + em_step(loglik, R, v) + separate" +
                               (", captured in one HIP graph and replayed" if args.graph else ""),
                       "launch_shapes": shapes})
    rec["eager_ms_per_step"] = eager_ms
    rec["roofline"] = roofline_entry(em_ms, flop_per_update(M) * updates, bytes_per_update(M) * F * N,
                                     load_traffic() if M == 4 else None,
                                     "em_kernel (all iterations of a call, one workgroup per frequency)")
    rec["in_run_baseline"] = {"kernel": "conv_em_kernel (conventional frame-wise EM, same workload)",
                              "kernel_ms_per_step": conv_ms, "updates_per_s": updates / (conv_ms * 1e-3),
                              "fastfca_kernel_speedup": conv_ms / em_ms,
                              "flagged_frequencies": int((conv_flags != 0).sum())}
    rec["loglik_first_last"] = [float(lls[0]), float(lls[-1])]
    rec["flagged_frequencies"] = int((flags != 0).sum())
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline([mx.y], L, args.F)
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
    bts = int(sum(bytes_per_update(int(m)) * F * int(n) for m, n in zip(Ms, Ns)))
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
    rec["roofline"] = roofline_entry(em_ms, flop, bts, None,
                                     "em_kernel, one launch per (M, frames-per-thread) group, groups concurrent")
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
    run_R, run_v = run.R, run.v
    run.close()
    updates = B * F * N * L
    rec = base_record(args, updates / (ms_step * 1e-3), ms_step,
                      {"workload": f"{B} array mixtures, M={M}, F={F}, N={N}, {L} EM iterations, "
                                   f"{'learned start with plain fallback' if learned else 'plain start'} "
                                   "(frames streamed from memory every pass)",
                       "mixtures": B, "M": M, "F": F, "N": N, "iterations": L,
                       "precision": "f32 per-bin arithmetic; f64 eigendecomposition and sums"})
    bts = bytes_per_update(M) * B * F * N * L   # streamed: y and v move every iteration
    rec["roofline"] = roofline_entry(em_ms, flop_per_update(M) * updates, bts, None,
                                     "em_stream_kernel (frames re-read every iteration)")
    rec["roofline"]["hbm_frac"] = rec["roofline"]["hbm_equivalent_GBps"] / PEAK_HBM_GBS
    rec["flagged_frequencies"] = int((flags != 0).sum())
    if learned:
        rec["learned_start"] = learned
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
    cores = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
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
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = {"value": len(idx) * N * L / cpu_s, "unit": "updates/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{len(idx)}/{F} frequencies x {N} frames of 1 mixture, {L} iterations "
                                         f"of the conventional FCA EM in FP64 ({cpu_s:.2f} s wall)"}
    return rec


def run_time_to_target(args):
    import numpy as np
    import torch
    from paper_1805_06572_amd import fca, learned_init, schedule, synth

    M, F, N, K, L = 4, 513, 1000, args.mixtures, args.iters
    widths = [int(h) for h in args.hidden.split(",")]
    ys = [synth.array_mixture_device(M, F, N, seed=3000 + k, ar1=True)[0] for k in range(K)]
    ys64 = [y.to(torch.complex128) for y in ys]
    torch.cuda.synchronize()

    # Plain FastFCA (plain start, FP64, one mixture at a time, L iterations)
    # defines each mixture's target: LL(theta^L), with a threshold at 99.9 % of
    # the rise from LL(theta^0).
    def one_at_a_time(yl, prec):
        out = []
        for y in yl:
            run = Runner(fca, [y], L, prec)
            step_ms, _ = run.timed(2, 1, separate=False)
            ll = run.ll.cpu().numpy()[0]
            last, _, _ = fca.fca_em_step(run.ctx, 0, want_R=False, want_v=False, allow_flags=True)
            out.append((step_ms, np.r_[ll, last.cpu().numpy()[0, 0]]))
            run.close()
        return out

    p64 = one_at_a_time(ys64, fca.FCA_FP64)
    targets = np.array([h[-1] for _, h in p64])
    thr = targets - 1e-3 * (targets - np.array([h[0] for _, h in p64]))

    def first_hit(h, t):
        hit = np.nonzero(np.asarray(h) >= t)[0]
        return int(hit[0]) if len(hit) else None

    def prorated(runs):
        its = [first_hit(h, thr[k]) for k, (_, h) in enumerate(runs)]
        ms = sum(step_ms * (L if it is None else it) / L for (step_ms, _), it in zip(runs, its))
        return ms, its

    plain64_ms, plain64_its = prorated(p64)
    plain32_ms, plain32_its = prorated(one_at_a_time(ys, fca.FCA_FP32_BULK))

    hit_rule = schedule.reached(thr)
    conv_rule = schedule.converged(1e-6)

    def stop(b, ll):
        return hit_rule(b, ll) or conv_rule(b, ll)

    mask = args.mask_sharpen if args.mask_sharpen > 0 else None

    def choice_iter(m):
        """Iterations before the starts are compared: 0 with the mask-based R
        (its LL(theta^0) already ranks the starts), 1 without (at theta^0 the
        plain start's equal powers look better than they are)."""
        if args.choice_iter >= 0:
            return args.choice_iter
        return 0 if m is not None else 1

    def batched(net, mask=None):
        """Wall time of one batched FP32 run from context-ready to every
        mixture stopped, with the learned start of `net` (or the plain start
        if None; with `mask`, the learned start's R from its masks sharpened
        by that exponent); warm: the same run once before, untimed."""
        res = None
        for rep in range(2):
            ctx = fca.fca_init_batch(ys, prec=fca.FCA_FP32_BULK)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            chosen, adv = None, np.zeros(len(ys), dtype=int)
            if net is not None:
                chosen, _, _, adv = learned_init.choose_starts(net, ctx, ys, choice_iter=choice_iter(mask),
                                                               mask_sharpen=mask)
            t2 = time.perf_counter()
            # stop checks: the mask start reaches the target in about 20
            # iterations, the other starts in 30 to 50 (each path at the
            # faster of these two chunkings, measured)
            chunks = (16, 4) if (net is not None and mask is not None) else (16, 8, 4)
            iters, hist = schedule.run_batch(ctx, 2 * L, chunks, stop)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            fca.fca_destroy(ctx)
            # a kept learned start enters the run `adv` iterations in
            res = ((t3 - t1) * 1e3, (t2 - t1) * 1e3, np.asarray(iters) + adv, hist, chosen, adv)
        return res

    bp_ms, _, bp_iters, bp_hist, _, _ = batched(None)
    bp_hits = [first_hit(h, thr[k]) for k, h in enumerate(bp_hist)]
    learned = {}
    for H in widths:
        t0 = time.perf_counter()
        net, _ = learned_init.train(M=M, F=F, steps=args.train_steps, batch=8192, seed=0, hidden=H,
                                    cosine=args.cosine)
        train_s = time.perf_counter() - t0
        bce, bce_const = learned_init.evaluate(net, n=65536, M=M, F=F)
        bl_ms, bl_init_ms, bl_iters, bl_hist, chosen, adv = batched(net, mask)
        bl_hits = [first_hit(h, thr[k]) for k, h in enumerate(bl_hist)]
        bl_hits = [None if h is None else int(h + a) for h, a in zip(bl_hits, adv)]
        extra = {}
        if mask is not None and H == widths[0]:
            # the same network without the mask-based R, for comparison
            nm_ms, nm_init_ms, nm_iters, nm_hist, nm_chosen, nm_adv = batched(net, None)
            nm_hits = [first_hit(h, thr[k]) for k, h in enumerate(nm_hist)]
            nm_hits = [None if h is None else int(h + a) for h, a in zip(nm_hits, nm_adv)]
            extra["without_mask_R"] = {
                "batched_learned_start_fp32_ms": nm_ms, "start_choice_ms": nm_init_ms,
                "speedup_vs_plain_fp64": plain64_ms / nm_ms, "mean_iterations_run": float(np.mean(nm_iters)),
                "mean_iterations_to_target": float(np.mean([h for h in nm_hits if h is not None])),
                "reached": sum(i is not None for i in nm_hits), "learned_start_chosen": int(np.sum(nm_chosen))}
        learned[H] = {
            "hidden": H, "batched_learned_start_fp32_ms": bl_ms, "start_choice_ms": bl_init_ms,
            "speedup_vs_plain_fp64": plain64_ms / bl_ms, "speedup_vs_plain_fp32": plain32_ms / bl_ms,
            "speedup_of_learned_start_in_batch": bp_ms / bl_ms,
            "mean_iterations_run": float(np.mean(bl_iters)),
            "iterations_to_target": bl_hits, "reached": sum(i is not None for i in bl_hits),
            "learned_start_chosen": int(np.sum(chosen)),
            "mlp_train_s": train_s, "mlp_train_steps": args.train_steps,
            "mlp_heldout_bce": bce, "constant_predictor_bce": bce_const,
            "mask_R": None if mask is None else {"sharpen": mask, "load": 1e-3}, **extra}
        net.close()
    head = learned[widths[0]]
    bl_ms = head["batched_learned_start_fp32_ms"]
    rec = base_record(args, K * F * N * head["mean_iterations_run"] / (bl_ms * 1e-3), bl_ms,
                      {"workload": f"time to target: {K} held-out array mixtures (AR(1) log-powers), M={M}, "
                                   f"F={F}, N={N}; target = LL of plain FastFCA (FP64, plain start) after "
                                   f"{L} iterations, reached at 99.9 % of its rise; learned start of hidden "
                                   f"width {widths[0]}" + ("" if mask is None else
                                                          f", R from its masks (sharpen {mask})"),
                       "mixtures": K, "M": M, "F": F, "N": N, "iterations": L, "hidden": widths[0]})
    rec["steps"], rec["warmup"] = 1, 1
    rec["time_to_target"] = {
        "plain_fastfca_fp64_one_at_a_time_ms": plain64_ms,
        "plain_fastfca_fp32_one_at_a_time_ms": plain32_ms,
        "batched_plain_start_fp32_ms": bp_ms,
        "batched_plain_mean_iterations_run": float(np.mean(bp_iters)),
        "iterations_to_target": {"plain_fp64": plain64_its, "plain_fp32": plain32_its,
                                 "batched_plain": bp_hits},
        "reached": {"plain_fp32": sum(i is not None for i in plain32_its),
                    "batched_plain": sum(i is not None for i in bp_hits)},
        "learned": [learned[H] for H in widths],
        "start_choice": f"per mixture, the start with the higher LL after {choice_iter(mask)} EM iteration(s) "
                        f"({choice_iter(None)} without the mask-based R; plain start as fallback); a kept "
                        "learned start continues from the iterate after the comparison; the learned start takes "
                        "R from its masks (fca_set_mask_covariances) unless --mask-sharpen 0",
        "stop_rule": "reached target, or LL rise below 1e-6 of the total (converged elsewhere), checked after "
                     "16 and then every 4 iterations with the mask-based start, after 16, 24 and then every 4 "
                     "iterations otherwise (each call reloads the frames: ~1 ms at 256 mixtures)"}
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="array", choices=["array", "batched", "large", "time-to-target"])
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--M", type=int, default=4)
    ap.add_argument("--F", type=int, default=513)
    ap.add_argument("--N", type=int, default=1000)
    ap.add_argument("--mixtures", type=int, default=256, help="time-to-target: held-out mixtures")
    ap.add_argument("--train-steps", type=int, default=None,
                    help="training steps of 8192 bins for the learned start (default: 20000 for "
                         "time-to-target, 2000 for the large workload)")
    ap.add_argument("--cosine", action="store_true", help="time-to-target: cosine-decayed training rate")
    ap.add_argument("--plain-large", dest="learned_large", action="store_false",
                    help="large workload: plain start only (no learned start)")
    ap.add_argument("--hidden", default="32,64,256",
                    help="time-to-target: hidden widths of the learned-start networks (the first one is the "
                         "headline)")
    ap.add_argument("--choice-iter", type=int, default=-1,
                    help="time-to-target: EM iterations after which the plain and learned starts are compared "
                         "(-1: 0 with the mask-based R, 1 without)")
    ap.add_argument("--mask-sharpen", type=float, default=3.0,
                    help="time-to-target: sharpening exponent of the masks that give the learned start its R "
                         "(0: plain R)")
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
              "time-to-target": run_time_to_target}[args.workload]
    print(json.dumps(runner(args)), flush=True)


if __name__ == "__main__":
    main()
