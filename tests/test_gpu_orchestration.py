"""GPU tests of the batched orchestration: launch shapes (128-thread
workgroups), the autotuner, concurrent launch groups and the captured step
(HIP graph), all through the C ABI and against the CPU oracle or the eager
path."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1805_06572_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def fca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_06572_amd import fca as mod
    mod.lib()
    return mod


def rel(a, b, axes):
    return np.sqrt((np.abs(a - b) ** 2).sum(axes)) / np.sqrt((np.abs(b) ** 2).sum(axes))


# mixed batch: several launch groups, ragged tails, one streamed mixture
SHAPES = [(2, 90), (4, 700), (3, 1000), (8, 300), (4, 2500), (6, 129)]


def batch(F=5, seed=700, dtype=np.complex128):
    mxs = [synth.random_mixture(M, F, N, seed + i) for i, (M, N) in enumerate(SHAPES)]
    return mxs, [torch.from_numpy(m.y.astype(dtype)).to(DEV) for m in mxs]


def test_128_thread_shape_matches_oracle(fca):
    """Every group that 128-thread workgroups can hold runs with them; FP64
    results match the oracle per mixture."""
    mxs, ys = batch()
    ctx = fca.fca_init_batch(ys, prec=fca.FCA_FP64)
    try:
        groups = fca.fca_launch_groups(ctx)
        changed = 0
        for g, info in enumerate(groups):
            if info["frames_per_thread"] != 0 and info["max_frames"] <= 1024:
                fca.fca_set_launch_shape(ctx, g, 128)
                changed += 1
            else:
                with pytest.raises(fca.FcaError):
                    fca.fca_set_launch_shape(ctx, g, 128)
        assert changed >= 4
        after = fca.fca_launch_groups(ctx)
        for info in after:
            if info["threads"] == 128:
                assert info["frames_per_thread"] * 128 >= info["max_frames"]
        ll, R, v = fca.fca_em_step(ctx, 6)
    finally:
        fca.fca_destroy(ctx)
    for k, mx in enumerate(mxs):
        S0, v0 = oracle.default_init(mx.y)
        S, vo, llo, fl = oracle.em(mx.y, S0, v0, 6, threads=8)
        assert not fl.any()
        assert rel(v[k].cpu().numpy(), vo, (-1,)).max() < 1e-10
        assert rel(R[k].cpu().numpy(), S, (-2, -1)).max() < 1e-10
        np.testing.assert_allclose(ll[k].cpu().numpy(), llo[:6].sum(1), rtol=1e-10)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_streamed_shape_for_every_group(fca, prec):
    """Every group switched to the streaming kernel: FP64 matches the oracle,
    FP32 matches the resident FP32 run within the float tolerance."""
    P = fca.FCA_FP64 if prec == "fp64" else fca.FCA_FP32_BULK
    mxs, ys = batch(dtype=np.complex128 if prec == "fp64" else np.complex64)
    ctx = fca.fca_init_batch(ys, prec=P)
    ref = fca.fca_init_batch(ys, prec=P)
    try:
        for g in range(len(fca.fca_launch_groups(ctx))):
            fca.fca_set_launch_shape(ctx, g, 256, streamed=True)
        assert all(info["frames_per_thread"] == 0 for info in fca.fca_launch_groups(ctx))
        with pytest.raises(fca.FcaError):
            fca.fca_set_launch_shape(ctx, 0, 128, streamed=True)
        ll, R, v = fca.fca_em_step(ctx, 6, allow_flags=True)
        llr, Rr, vr = fca.fca_em_step(ref, 6, allow_flags=True)
    finally:
        fca.fca_destroy(ctx)
        fca.fca_destroy(ref)
    if prec == "fp64":
        for k, mx in enumerate(mxs):
            S0, v0 = oracle.default_init(mx.y)
            S, vo, llo, fl = oracle.em(mx.y, S0, v0, 6, threads=8)
            assert rel(v[k].cpu().numpy(), vo, (-1,)).max() < 1e-10
            assert rel(R[k].cpu().numpy(), S, (-2, -1)).max() < 1e-10
            np.testing.assert_allclose(ll[k].cpu().numpy(), llo[:6].sum(1), rtol=1e-10)
    else:
        for k in range(len(ys)):
            assert rel(v[k].double().cpu().numpy(), vr[k].double().cpu().numpy(), (-1,)).max() < 1e-4


def test_autotune_restores_state_and_keeps_results(fca):
    mxs, ys = batch(dtype=np.complex64)
    a = fca.fca_init_batch(ys, prec=fca.FCA_FP32_BULK)
    b = fca.fca_init_batch(ys, prec=fca.FCA_FP32_BULK)
    try:
        fca.fca_em_step(a, 2, allow_flags=True)
        fca.fca_em_step(b, 2, allow_flags=True)
        _, R0, v0 = fca.fca_em_step(a, 0, allow_flags=True)
        fca.fca_autotune(a, 3)
        _, R1, v1 = fca.fca_em_step(a, 0, allow_flags=True)
        for k in range(len(ys)):                     # the trials left no trace
            assert torch.equal(R0[k], R1[k]) and torch.equal(v0[k], v1[k])
        shapes = fca.fca_launch_groups(a)
        assert all(s["threads"] in (128, 256) for s in shapes)
        lla, Ra, va = fca.fca_em_step(a, 5, allow_flags=True)
        llb, Rb, vb = fca.fca_em_step(b, 5, allow_flags=True)
        np.testing.assert_allclose(lla.cpu().numpy(), llb.cpu().numpy(), rtol=1e-5)
        for k in range(len(ys)):
            assert rel(va[k].double().cpu().numpy(), vb[k].double().cpu().numpy(), (-1,)).max() < 1e-4
    finally:
        fca.fca_destroy(a)
        fca.fca_destroy(b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replays_equal_the_eager_step(fca, prec):
    """reset + L iterations + R, v, x out, captured once and replayed three
    times with eager work in between: every replay equals the eager step
    bit for bit."""
    P = fca.FCA_FP64 if prec == "fp64" else fca.FCA_FP32_BULK
    _, ys = batch(dtype=np.complex128 if prec == "fp64" else np.complex64)
    L = 7
    ctx = fca.fca_init_batch(ys, prec=P)
    try:
        ll_e, R_e, v_e = fca.fca_em_step(ctx, L, allow_flags=True)
        x_e = fca.fca_separate(ctx)
        g = fca.fca_graph_capture(ctx, L, with_reset=True, want_x=True)
        for rep in range(3):
            fca.fca_graph_launch(g, 1, allow_flags=True)
            assert torch.equal(g.loglik, ll_e)
            assert torch.equal(g.R, torch.cat([r.reshape(-1) for r in R_e]))
            assert torch.equal(g.v, torch.cat([t.reshape(-1) for t in v_e]))
            assert torch.equal(g.x, torch.cat([t.reshape(-1) for t in x_e]))
            # eager work between replays on the same context and stream
            fca.fca_reset(ctx)
            fca.fca_em_step(ctx, 2, allow_flags=True)
            torch.cuda.synchronize()
        fca.fca_graph_launch(g, 4, allow_flags=True)     # back-to-back replays
        assert torch.equal(g.loglik, ll_e)
    finally:
        fca.fca_destroy(ctx)


def test_graph_with_inactive_mixture_and_stale_shape(fca):
    _, ys = batch()
    ctx = fca.fca_init_batch(ys, prec=fca.FCA_FP64)
    ref = fca.fca_init_batch(ys, prec=fca.FCA_FP64)
    try:
        fca.fca_set_active(ctx, 1, False)
        g = fca.fca_graph_capture(ctx, 4, with_reset=True)
        fca.fca_graph_launch(g, 2)
        ll_r, R_r, v_r = fca.fca_em_step(ref, 4)
        ll = g.loglik.cpu().numpy()
        assert np.isnan(ll[1]).all()
        others = [k for k in range(len(ys)) if k != 1]
        np.testing.assert_array_equal(ll[others], ll_r.cpu().numpy()[others])
        # mixture 1 was reset by the replay but not iterated: its v is the plain start
        fca.fca_reset(ref)
        _, _, v_start = fca.fca_em_step(ref, 0)
        n0 = sum(2 * ctx.F * n for n in ctx.Ns[:1])
        n1 = n0 + 2 * ctx.F * ctx.Ns[1]
        assert torch.equal(g.v[n0:n1], v_start[1].reshape(-1))
        fca.fca_set_active(ctx, 1, True)               # activity changed since the capture
        with pytest.raises(fca.FcaError) as e:
            fca.fca_graph_launch(g, 1)
        assert e.value.status == fca.FCA_E_STATE
        g2 = fca.fca_graph_capture(ctx, 4, with_reset=True)
        fca.fca_graph_launch(g2, 1)
        np.testing.assert_array_equal(g2.loglik.cpu().numpy(), ll_r.cpu().numpy())
    finally:
        fca.fca_destroy(ctx)
        fca.fca_destroy(ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_resume_from_exported_parameters(fca, prec):
    """Checkpoint and resume: 6 iterations, export (R, v), start a second
    context from them with fca_set_start and run 4 more; the result equals
    10 straight iterations. The resumed context rebuilds its basis from R
    (another eigendecomposition of the same pencil), so the agreement is to
    rounding, not bitwise: relative 1e-9 in FP64, 1e-4 in FP32 bulk."""
    P = fca.FCA_FP64 if prec == "fp64" else fca.FCA_FP32_BULK
    tol = 1e-9 if prec == "fp64" else 1e-4
    mxs, ys = batch(dtype=np.complex128 if prec == "fp64" else np.complex64)
    straight = fca.fca_init_batch(ys, prec=P)
    resumed = fca.fca_init_batch(ys, prec=P)
    try:
        ll, R, v = fca.fca_em_step(straight, 10, allow_flags=True)
        _, R6, v6 = fca.fca_em_step(resumed, 6, allow_flags=True)
        for k in range(len(ys)):
            fca.fca_set_start(resumed, k, R6[k].clone(), v6[k].clone())
        ll2, R2, v2 = fca.fca_em_step(resumed, 4, allow_flags=True)
    finally:
        fca.fca_destroy(straight)
        fca.fca_destroy(resumed)
    for k in range(len(ys)):
        assert rel(v2[k].double().cpu().numpy(), v[k].double().cpu().numpy(), (-1,)).max() < tol
        assert rel(R2[k].cpu().numpy(), R[k].cpu().numpy(), (-2, -1)).max() < tol
        np.testing.assert_allclose(ll2[k].cpu().numpy(), ll[k, 6:].cpu().numpy(), rtol=tol)


def test_invalid_arguments_are_rejected_and_leave_the_context_usable(fca):
    """Host-side argument checks of the ABI: FCA_E_ARG (or FCA_E_STATE) and
    no change to a live context."""
    import ctypes
    L = fca.lib()
    mx = synth.random_mixture(2, 3, 40, 5)
    y = torch.from_numpy(mx.y).to(DEV)

    def init_status(**over):
        p = fca.fca_problem(M=2, F=3, N=40, prec=fca.FCA_FP64, y=y.data_ptr(), y_stride_f=y.stride(0),
                            y_stride_n=y.stride(1), y_stride_m=y.stride(2), R0=None, v0=None, stream=None)
        for k, val in over.items():
            setattr(p, k, val)
        h = ctypes.c_void_p()
        st = L.fca_init(ctypes.byref(p), ctypes.byref(h))
        if h.value:
            L.fca_destroy(h)
        return st, h.value

    st, h = init_status()
    assert st == fca.FCA_OK and h is not None
    for bad in ({"M": 0}, {"M": 9}, {"F": 0}, {"N": 0}, {"prec": 7}, {"y": None}, {"y_stride_n": -1}):
        st, h = init_status(**bad)
        assert st == fca.FCA_E_ARG and h is None, bad
    with pytest.raises(fca.FcaError) as e:          # batch members must share F
        fca.fca_init_batch([y, y[:2]], prec=fca.FCA_FP64)
    assert e.value.status == fca.FCA_E_ARG

    ctx = fca.fca_init(y, prec=fca.FCA_FP64)
    try:
        ll0, _, _ = fca.fca_em_step(ctx, 3, want_R=False, want_v=False)
        fca.fca_reset(ctx)
        h = ctx.handle
        assert L.fca_em_step(h, -1, None, None, None) == fca.FCA_E_ARG
        assert L.fca_set_start(h, 1, None, None) == fca.FCA_E_ARG
        assert L.fca_set_active(h, -1, 0) == fca.FCA_E_ARG
        assert L.fca_set_launch_shape(h, 5, 128, 0) == fca.FCA_E_ARG
        assert L.fca_set_launch_shape(h, 0, 64, 0) == fca.FCA_E_ARG
        assert L.fca_graph_launch(h, 1) == fca.FCA_E_STATE
        host_ll = np.zeros((1, 3))
        assert L.fca_graph_capture(h, 3, 1, host_ll.ctypes.data, None, None, None) == fca.FCA_E_ARG
        assert L.fca_em_step(None, 1, None, None, None) == fca.FCA_E_ARG
        host = np.zeros((1, 2, 2), np.complex128)
        flags = np.zeros(1, np.int32)
        lam = np.zeros(2)
        assert L.fca_gevd(2, 1, host.ctypes.data, host.ctypes.data, host.ctypes.data, lam.ctypes.data,
                          flags.ctypes.data, None) == fca.FCA_E_ARG
        ll1, _, _ = fca.fca_em_step(ctx, 3, want_R=False, want_v=False)
        assert torch.equal(ll0, ll1)
    finally:
        fca.fca_destroy(ctx)


def test_batched_workload_full_size_sampled_against_oracle(fca):
    """The 64-mixture uneven batch of the benchmark (same draws, autotuned
    shapes, concurrent groups, captured step), 50 iterations: for one mixture
    of each microphone count, four frequencies against the oracle run from
    the same plain start (computed from the whole mixture)."""
    rng = np.random.default_rng(2)
    B, F, L = 64, 513, 50
    Ns = rng.integers(200, 2001, size=B)
    Ms = rng.choice([2, 4, 8], size=B)
    gen = [synth.array_mixture_device(int(Ms[b]), F, int(Ns[b]), seed=1000 + b) for b in range(B)]
    ys = [g[0] for g in gen]
    ctx = fca.fca_init_batch(ys, prec=fca.FCA_FP32_BULK)
    try:
        fca.fca_autotune(ctx, 3)
        g = fca.fca_graph_capture(ctx, L, with_reset=True)
        fca.fca_graph_launch(g, 1, allow_flags=True)
        ll_gpu = g.loglik.cpu().numpy()
        flags = fca.fca_status_per_freq(ctx)
        v_off = np.cumsum([0] + [2 * F * int(n) for n in Ns])
        checked = 0
        for M in (2, 4, 8):
            b = int(np.nonzero(Ms == M)[0][0])
            N = int(Ns[b])
            y = ys[b].cpu().numpy().astype(np.complex128)
            kappa = synth.condition_numbers(gen[b][2])
            idx = np.nonzero(kappa <= 1e3)[0]
            idx = idx[np.linspace(0, len(idx) - 1, 4).round().astype(int)]
            S0, v0 = oracle.default_init(y)
            S, v, ll, fl = oracle.em(np.ascontiguousarray(y[idx]), np.ascontiguousarray(S0[:, idx]),
                                     np.ascontiguousarray(v0[:, idx]), L, threads=8)
            gv = g.v[v_off[b]:v_off[b + 1]].view(2, F, N)[:, idx].double().cpu().numpy()
            ok = (fl == 0) & (flags[b, idx] == 0)
            assert rel(gv, v, (-1,))[:, ok].max() < 1e-4, (M, rel(gv, v, (-1,)))
            checked += int(ok.sum())
            assert np.all(np.isfinite(ll_gpu[b])) and np.all(np.diff(ll_gpu[b]) > -1e-4 * np.abs(ll_gpu[b][1:]))
        assert checked >= 10
    finally:
        fca.fca_destroy(ctx)
