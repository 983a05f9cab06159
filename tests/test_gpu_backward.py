"""GPU parity of the adjoint (sos_filt_backward) against the FP64 oracle
adjoint, which is itself pinned to dense matrix transposes and central
finite differences on the CPU (test_oracle.py).

Tolerances:
* FP64 in/out, against the oracle adjoint in extended precision (long
  double): dL/dx within max(1e-12, 4 e) relative RMS and dL/dsos within
  max(1e-10, 4 e) of the largest entry of its row, e being the FP64 oracle
  adjoint's own error against the same reference.  The adjoint runs the
  all-pole step before the numerator (mu = A^{-T} lambda, then B^T mu), so
  strongly attenuating cascades cancel large intermediates: on K = 8 draws the
  FP64 oracle itself is ~1e-12 (dL/dx) and ~3e-11 (dL/dsos) off.
* FP32 in/out: dL/dx within 1e-6 relative RMS (FP32 output rounding);
  dL/dsos within 1e-9 of the row's largest entry (FP64 arithmetic, and FP64
  section outputs whether saved or recomputed; the inputs x and dL/dy are
  exact in both).
"""
import numpy as np
import pytest

import oracle
from paper_2607_14054_amd import sosfilt as S
from paper_2607_14054_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def row_err(g, ref):
    scale = np.maximum(np.max(np.abs(ref), axis=1, keepdims=True), 1e-300)
    return float(np.max(np.abs(g - ref) / scale))


def check_f64(x, sos, g, gx, gs, tag=""):
    """GPU adjoint against the extended-precision oracle adjoint, bounded by
    the FP64 oracle adjoint's own error."""
    lx, ls = oracle.sosfilt_backward_ld(x, sos, g)
    ox, os_ = oracle.sosfilt_backward(x, sos, g)
    ex, es = oracle.rel_rms(gx, lx), row_err(gs, ls)
    ox_e, os_e = oracle.rel_rms(ox, lx), row_err(os_, ls)
    print("%s gx err=%.2e (oracle %.2e) gsos err=%.2e (oracle %.2e)" % (tag, ex, ox_e, es, os_e))
    assert ex <= max(1e-12, 4 * ox_e)
    assert es <= max(1e-10, 4 * os_e)


def run_backward(sos, x_np, g_np, **kw):
    io = "f64" if x_np.dtype == np.float64 else "f32"
    p = S.Plan(sos, io_dtype=io, **kw)
    x = torch.from_numpy(x_np).to(DEV)
    g = torch.from_numpy(g_np).to(DEV)
    gx, gs = S.filt_backward(p, x, g)
    torch.cuda.synchronize()
    return gx.cpu().numpy(), gs.cpu().numpy()


@pytest.mark.parametrize("adjoint", ["save", "recompute"])
@pytest.mark.parametrize("n", [1, 2, 17, 255, 256, 257, 5000, 70001, 2 ** 20 + 3])
@pytest.mark.parametrize("K", [1, 3, 8])
def test_backward_f64_matches_oracle_adjoint(n, K, adjoint):
    sos = W.make_sos(K, 0.5, 0.95, 40 + K)
    x = W.make_signal(n, 41, np.float64)
    g = W.grad_seed_signal(n, 41, np.float64)
    gx, gs = run_backward(sos, x, g, adjoint=adjoint)
    check_f64(x, sos, g, gx, gs, "n=%d K=%d %s" % (n, K, adjoint))


@pytest.mark.parametrize("io", ["f64", "f32"])
@pytest.mark.parametrize("K", [2, 16])
def test_backward_recompute_equals_saved_outputs(io, K):
    """The two adjoint modes (every section output kept in FP64, or the
    section inputs recomputed from group checkpoints) give the same
    gradients to rounding, with poles up to r = 0.99, and the oracle's."""
    dt = np.float64 if io == "f64" else np.float32
    n = 3 * 2 ** 16 + 1001
    sos = W.make_sos(K, 0.6, 0.99, 140 + K)
    x = W.make_signal(n, 141, dt)
    g = W.grad_seed_signal(n, 141, dt)
    rx, rs = run_backward(sos, x, g, adjoint="recompute")
    sx, ss = run_backward(sos, x, g, adjoint="save")
    assert oracle.rel_rms(rx, sx) < (1e-12 if io == "f64" else 1e-6)
    assert row_err(rs, ss) < 1e-10
    if io == "f64":
        check_f64(x, sos, g, rx, rs, "recompute K=%d" % K)


def test_backward_mode_choice_and_workspace():
    """Automatic mode by the measured cost model: recompute (checkpoints:
    2K + 2 doubles per 256-sample group, and for K >= 8 one kept section
    input, a double per sample) up to K = 40 with FP32 I/O and K = 31 with
    FP64 I/O, saved outputs above (K doubles per sample); both flags
    together are rejected."""
    n = 2 ** 20
    for io, cases in (("f32", ((1, True), (4, True), (8, True), (17, True), (18, True), (40, True), (41, False),
                               (48, False))),
                      ("f64", ((1, True), (8, True), (23, True), (31, True), (32, False), (40, False)))):
        for K, rc in cases:
            sos = W.make_sos(K, 0.5, 0.95, 150 + K)
            auto = S.Plan(sos, io_dtype=io).backward_workspace_size(n)
            save = S.Plan(sos, io_dtype=io, adjoint="save").backward_workspace_size(n)
            rec = S.Plan(sos, io_dtype=io, adjoint="recompute").backward_workspace_size(n)
            assert save >= K * n * 8
            kept = 8 * (n + 512) if K >= 8 else 0
            assert rec < (2 * K + 2) * 8 * (n // 256 + 2) + kept + save - K * n * 8
            assert (rec >= 8 * n) == (K >= 8)
            assert auto == (rec if rc else save), (io, K)
    import ctypes
    s2 = np.ascontiguousarray(W.make_sos(2, 0.5, 0.9, 1))
    o = S._Opts(S.SOS_F32, S.SOS_F64, S.SOS_AUTO, 0, 16, 0, S.SOS_FLAG_ADJ_SAVE | S.SOS_FLAG_ADJ_RECOMPUTE)
    h = ctypes.c_void_p()
    rc = S.lib().sos_plan(s2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2, ctypes.byref(o), ctypes.byref(h))
    assert rc == S.SOS_E_ARG and not h.value


def test_backward_f32_adjoint_config_channel():
    """One channel of the adjoint workload: 2^18 FP32 samples, K = 8,
    r in [0.5, 0.95], g ~ N(0, 1) with seed + 2."""
    c = W.CONFIGS["grad"]
    sos = W.make_sos(c.K, c.r_lo, c.r_hi, c.seed)
    x = W.make_signal(c.n, c.seed, np.float32)
    g = W.grad_seed_signal(c.n, c.seed, np.float32)
    gx, gs = run_backward(sos, x, g)
    rx, rs = oracle.sosfilt_backward(x.astype(np.float64), sos, g.astype(np.float64))
    ex, es = oracle.rel_rms(gx, rx), row_err(gs, rs)
    print("f32 adjoint: gx rel_rms=%.2e gsos row err=%.2e" % (ex, es))
    assert ex < 1e-6
    assert es < 1e-9


@pytest.mark.parametrize("solver,N,L", [("cr", 64, 16), ("ph", 8, 16), ("phd", 32, 16), ("ph", 4, 16),
                                         ("cr", 4, 16), ("auto", 128, 16), ("ph", 1024, 16), ("ph", 16, 64)])
def test_backward_independent_of_forward_solver(solver, N, L):
    """The adjoint runs on its own 16-block sub-plan: the same gradients
    whatever the forward plan's solver, width (N = 4 .. 1024) or block
    size."""
    sos = W.make_sos(4, 0.5, 0.95, 44)
    x = W.make_signal(30001, 45, np.float64)
    g = W.grad_seed_signal(30001, 45, np.float64)
    gx, gs = run_backward(sos, x, g, compute_dtype="f64", solver=solver, N=N, L=L)
    check_f64(x, sos, g, gx, gs, solver)


def test_backward_unfactored_b0_and_a0():
    sos = W.make_sos(3, 0.5, 0.95, 46)
    sos[1, 0:3] = [0.0, 0.5, -0.25]      # b0 = 0: no factoring
    sos[2] *= 2.5                        # a0 != 1
    x = W.make_signal(20000, 47, np.float64)
    g = W.grad_seed_signal(20000, 47, np.float64)
    gx, gs = run_backward(sos, x, g)
    check_f64(x, sos, g, gx, gs, "unfactored")


def test_backward_central_finite_differences_on_gpu_forward():
    """dL/dsos from the adjoint against FP64 central differences of
    L = sum(y * g), y from the GPU forward, on a 2^10-sample subset."""
    n = 2 ** 10
    sos = W.make_sos(2, 0.5, 0.9, 48)
    x = W.make_signal(n, 49, np.float64)
    g = W.grad_seed_signal(n, 49, np.float64)
    _, gs = run_backward(sos, x, g)
    xt = torch.from_numpy(x).to(DEV)

    def loss(s):
        y = S.filt(S.Plan(s, io_dtype="f64", compute_dtype="f64", solver="ph", N=8), xt)
        return float(np.dot(y.cpu().numpy(), g))

    fd = np.zeros_like(sos)
    for k in range(sos.shape[0]):
        for j in range(6):
            h = 1e-6 * max(abs(sos[k, j]), 1e-3)
            sp, sm = sos.copy(), sos.copy()
            sp[k, j] += h
            sm[k, j] -= h
            fd[k, j] = (loss(sp) - loss(sm)) / (2 * h)
    err = row_err(gs, fd)
    print("finite differences: row err %.2e" % err)
    assert err < 1e-6


@pytest.mark.parametrize("adjoint", ["save", "recompute"])
def test_backward_finite_differences_differentiation_workload(adjoint):
    """The differentiation workload's own cascade (channel 0: K = 8, pole
    radius U[0.5, 0.95], its float32 input and upstream gradient), on its
    first 2^10 samples: all 48 coefficient gradients of the adjoint, in
    both modes, against FP64 central differences of L = sum(y * g) with y
    from the GPU forward.  The differences themselves are good to about
    3e-7 of a row's largest entry here: the five-point stencil's h^4 term
    and the forward's FP64 rounding divided by h balance near h = 1e-5 of
    the coefficient (the two-point stencil's h^2 term alone reaches ~1e-6
    at these poles).  The adjoint's own error against the oracle adjoint is
    checked to 1e-10 first."""
    cfg = W.CONFIGS["grad"]
    n = 2 ** 10
    sos = W.make_sos(cfg.K, cfg.r_lo, cfg.r_hi, cfg.seed)
    x = W.make_signal(cfg.n, cfg.seed, np.float32)[:n].astype(np.float64)
    g = W.grad_seed_signal(cfg.n, cfg.seed, np.float32)[:n].astype(np.float64)
    gx, gs = run_backward(sos, x, g, adjoint=adjoint)
    check_f64(x, sos, g, gx, gs, "differentiation workload, " + adjoint)
    xt = torch.from_numpy(x).to(DEV)

    def loss(s):
        y = S.filt(S.Plan(s, io_dtype="f64", compute_dtype="f64", solver="ph", N=8), xt)
        return float(np.dot(y.cpu().numpy(), g))

    def at(k, j, d):
        s_ = sos.copy()
        s_[k, j] += d
        return loss(s_)

    fd = np.zeros_like(sos)
    for k in range(sos.shape[0]):
        for j in range(6):
            h = 1e-5 * max(abs(sos[k, j]), 1e-3)
            fd[k, j] = (at(k, j, -2 * h) - 8 * at(k, j, -h) + 8 * at(k, j, h) - at(k, j, 2 * h)) / (12 * h)
    err = row_err(gs, fd)
    print("finite differences, K = 8: row err %.2e" % err)
    assert err < 1e-6


def test_autograd_function_gradcheck():
    from paper_2607_14054_amd.autograd import SosFilt
    sos = torch.tensor(W.make_sos(2, 0.5, 0.9, 50), dtype=torch.float64, requires_grad=True)
    x = torch.tensor(W.make_signal(300, 51, np.float64), device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, b: SosFilt.apply(a, b, 8, "ph"), (x, sos),
                                    eps=1e-6, atol=1e-7, rtol=1e-5)


def test_zero_length_writes_zero_gradient():
    p = S.Plan(W.make_sos(3, 0.5, 0.9, 52), io_dtype="f32")
    x = torch.zeros(0, dtype=torch.float32, device=DEV)
    gx, gs = S.filt_backward(p, x, torch.zeros_like(x))
    torch.cuda.synchronize()
    assert gx.numel() == 0 and torch.all(gs == 0)


def test_backward_bad_arguments():
    import ctypes
    lib = S.lib()
    p = S.Plan(W.make_sos(2, 0.5, 0.9, 53), io_dtype="f32")
    x = torch.zeros(8192, dtype=torch.float32, device=DEV)
    gs = torch.zeros((2, 6), dtype=torch.float64, device=DEV)
    ws = torch.zeros(lib.sos_backward_workspace_size(p.handle, 4096) + 16, dtype=torch.uint8, device=DEV)
    vp = ctypes.c_void_p
    # gx overlapping x
    rc = lib.sos_filt_backward(p.handle, vp(x.data_ptr()), vp(x.data_ptr() + 16384), vp(x.data_ptr() + 64),
                               vp(gs.data_ptr()), 4096, vp(ws.data_ptr()), None)
    assert rc == S.SOS_E_ARG
    # no workspace
    rc = lib.sos_filt_backward(p.handle, vp(x.data_ptr()), vp(x.data_ptr() + 16384), vp(x.data_ptr() + 8192),
                               vp(gs.data_ptr()), 2048, None, None)
    assert rc == S.SOS_E_ARG
    host = S.Plan(W.make_sos(2, 0.5, 0.9, 53), host_only=True)
    assert lib.sos_backward_workspace_size(host.handle, 100) == 0


def test_batched_adjoint_mode_choice():
    """One adjoint mode per batch: saved outputs if any plan asks for them,
    else recompute if any asks for it, else the cheaper one over the batch's
    samples (K = 2 and 4 channels recompute; a batch dominated by K = 48
    keeps the outputs, one dominated by K = 4 recomputes).  The workspace
    shows the mode: K doubles per sample for saved outputs, group
    checkpoints and one kept section input (K >= 4) for recompute."""
    def ws(Ks, modes, lengths=(5000, 70001)):
        plans = [S.Plan(W.make_sos(k, 0.5, 0.95, 190 + i), io_dtype="f32", adjoint=m)
                 for i, (k, m) in enumerate(zip(Ks, modes))]
        return S.Batch(plans, list(lengths)).backward_workspace_size()
    saved_bytes = 8 * (2 * 5000 + 4 * 70001)
    assert ws([2, 4], ["auto", "auto"]) < saved_bytes / 3
    assert ws([2, 4], ["auto", "save"]) >= saved_bytes
    assert ws([2, 4], ["recompute", "auto"]) < saved_bytes / 3
    assert ws([2, 4], ["recompute", "save"]) >= saved_bytes
    assert ws([2, 48], ["auto", "auto"]) >= 8 * (2 * 5000 + 48 * 70001)
    assert ws([48, 4], ["auto", "auto"], (1000, 200000)) < 8 * (48 * 1000 + 4 * 200000) / 3


@pytest.mark.parametrize("adjoint", ["save", "recompute"])
@pytest.mark.parametrize("io", ["f64", "f32"])
def test_batched_adjoint_matches_oracle(io, adjoint):
    """sos_filt_backward_batched on ragged channels (dense packing, so f32
    channels also start off 16-byte boundaries), K mixed."""
    dt = np.float64 if io == "f64" else np.float32
    lengths = [0, 1, 17, 255, 5000, 70001, 2 ** 18 + 5]
    Ks = [3, 8, 1, 16, 5, 8, 2]
    sos = [W.make_sos(k, 0.5, 0.95, 70 + c) for c, k in enumerate(Ks)]
    plans = [S.Plan(s_, io_dtype=io, compute_dtype="f64", N=32, adjoint=adjoint) for s_ in sos]
    b = S.Batch(plans, lengths)
    xs = [W.make_signal(n, 71 + c, dt) for c, n in enumerate(lengths)]
    gs = [W.grad_seed_signal(n, 71 + c, dt) for c, n in enumerate(lengths)]
    xb = np.zeros(b.total, dt)
    gb = np.zeros(b.total, dt)
    for c in range(len(lengths)):
        o = b.offsets[c]
        xb[o:o + lengths[c]] = xs[c]
        gb[o:o + lengths[c]] = gs[c]
    gx, gsos, first = S.filt_backward_batched(b, torch.from_numpy(xb).to(DEV), torch.from_numpy(gb).to(DEV))
    torch.cuda.synchronize()
    gx = gx.cpu().numpy()
    gsos = gsos.cpu().numpy()
    for c in range(len(lengths)):
        o, n, K = b.offsets[c], lengths[c], Ks[c]
        g_c = gsos[first[c]:first[c] + K]
        if n == 0:
            assert np.all(g_c == 0)
            continue
        x64, g64 = xs[c].astype(np.float64), gs[c].astype(np.float64)
        if io == "f64":
            check_f64(x64, sos[c], g64, gx[o:o + n], g_c, "batched c=%d" % c)
        else:
            rx, rs = oracle.sosfilt_backward(x64, sos[c], g64)
            assert oracle.rel_rms(gx[o:o + n], rx) < 1e-6, c
            assert row_err(g_c, rs) < 1e-9, c


@pytest.mark.parametrize("adjoint", ["save", "recompute"])
@pytest.mark.parametrize("io", ["f32", "f64"])
def test_batched_adjoint_shifted_starts_keep_neighbours(io, adjoint):
    """Channels starting 1..V-1 samples past a 16-byte boundary (V samples
    per 16 bytes) with gaps of 1..3 samples between them, lengths around
    whole groups of the adjoint tiles: dL/dx and dL/dsos match the oracle
    and the gap samples of gx keep their value."""
    dt = np.float64 if io == "f64" else np.float32
    V = 16 // np.dtype(dt).itemsize
    G = 256                                       # adjoint group: N = 16, 16 lanes
    lengths, offsets, pos = [], [], 0
    for i, n in enumerate([1, 2, 3, G - 3, G - 2, G - 1, G, G + 1, 2 * G - 1, 3 * G + 5, 5000, 70001]):
        s_ = 1 + i % (V - 1) if V > 2 else 1
        pos = (pos + V - 1) // V * V + s_
        offsets.append(pos)
        lengths.append(n)
        pos += n + 1 + i % 3
    Ks = [1 + (5 * c) % 9 for c in range(len(lengths))]
    sos = [W.make_sos(k, 0.5, 0.95, 170 + c) for c, k in enumerate(Ks)]
    plans = [S.Plan(s_, io_dtype=io, compute_dtype="f64", N=32, adjoint=adjoint) for s_ in sos]
    b = S.Batch(plans, lengths, offsets=offsets)
    xs = [W.make_signal(n, 171 + c, dt) for c, n in enumerate(lengths)]
    gs = [W.grad_seed_signal(n, 171 + c, dt) for c, n in enumerate(lengths)]
    xb = np.zeros(b.total, dt)
    gb = np.zeros(b.total, dt)
    for c, o in enumerate(offsets):
        xb[o:o + lengths[c]] = xs[c]
        gb[o:o + lengths[c]] = gs[c]
    gx0 = torch.full((b.total,), -3.0, dtype=torch.float32 if io == "f32" else torch.float64, device=DEV)
    gx, gsos, first = S.filt_backward_batched(b, torch.from_numpy(xb).to(DEV), torch.from_numpy(gb).to(DEV),
                                              gx=gx0)
    torch.cuda.synchronize()
    gx = gx.cpu().numpy()
    gsos = gsos.cpu().numpy()
    mask = np.ones(b.total, bool)
    for c, o in enumerate(offsets):
        n, K = lengths[c], Ks[c]
        mask[o:o + n] = False
        g_c = gsos[first[c]:first[c] + K]
        x64, g64 = xs[c].astype(np.float64), gs[c].astype(np.float64)
        if io == "f64":
            check_f64(x64, sos[c], g64, gx[o:o + n], g_c, "shifted c=%d" % c)
        else:
            rx, rs = oracle.sosfilt_backward(x64, sos[c], g64)
            assert oracle.rel_rms(gx[o:o + n], rx) < 1e-6, (c, n, o % V)
            assert row_err(g_c, rs) < 1e-9, (c, n, o % V)
    assert np.all(gx[mask] == -3.0)


def test_batched_adjoint_equals_single_channel_adjoint():
    """Each channel of the batched adjoint equals sos_filt_backward on that
    channel alone to rounding (the tiles differ)."""
    lengths = [3000, 40000, 9000]
    sos = [W.make_sos(4, 0.5, 0.95, 80), W.make_sos(6, 0.5, 0.95, 81), W.make_sos(9, 0.5, 0.95, 83)]
    plans = [S.Plan(s_, io_dtype="f64", compute_dtype="f64", N=32) for s_ in sos]
    b = S.Batch(plans, lengths)
    xs = [W.make_signal(n, 82 + c, np.float64) for c, n in enumerate(lengths)]
    gs = [W.grad_seed_signal(n, 82 + c, np.float64) for c, n in enumerate(lengths)]
    xb = torch.from_numpy(np.concatenate(xs)).to(DEV)
    gb = torch.from_numpy(np.concatenate(gs)).to(DEV)
    gx, gsos, first = S.filt_backward_batched(b, xb, gb)
    for c in range(3):
        sx, ss = S.filt_backward(plans[c], torch.from_numpy(xs[c]).to(DEV), torch.from_numpy(gs[c]).to(DEV))
        o = b.offsets[c]
        assert oracle.rel_rms(gx[o:o + lengths[c]].cpu().numpy(), sx.cpu().numpy()) < 1e-13
        assert row_err(gsos[first[c]:first[c] + plans[c].K].cpu().numpy(), ss.cpu().numpy()) < 1e-12


@pytest.mark.parametrize("K", [6, 10])
@pytest.mark.parametrize("adjoint", ["save", "recompute"])
def test_adjoint_graph_replays_match_eager(adjoint, K):
    """sos_filt_backward (three kernels, caller workspace) captured in a HIP
    graph: every replay equals the eager call bit for bit (K = 10: the
    recompute forward also keeps section 5's input)."""
    import ctypes
    lib = S.lib()
    sos = W.make_sos(K, 0.5, 0.95, 92)
    n = 200003
    p = S.Plan(sos, io_dtype="f32", compute_dtype="f64", N=32, adjoint=adjoint)
    x = torch.from_numpy(W.make_signal(n, 93, np.float32)).to(DEV)
    g = torch.from_numpy(W.grad_seed_signal(n, 93, np.float32)).to(DEV)
    gx = torch.empty_like(x)
    gs = torch.empty((K, 6), dtype=torch.float64, device=DEV)
    ws = torch.empty(lib.sos_backward_workspace_size(p.handle, n), dtype=torch.uint8, device=DEV)
    vp = ctypes.c_void_p

    def call(stream):
        rc = lib.sos_filt_backward(p.handle, vp(x.data_ptr()), vp(g.data_ptr()), vp(gx.data_ptr()),
                                   vp(gs.data_ptr()), n, vp(ws.data_ptr()), vp(stream.cuda_stream))
        assert rc == 0

    call(torch.cuda.current_stream())
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=torch.cuda.Stream()):
        call(torch.cuda.current_stream())
    for rep in range(3):
        g.copy_(torch.from_numpy(W.grad_seed_signal(n, 94 + rep, np.float32)).to(DEV))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got_x, got_s = gx.clone(), gs.clone()
        call(torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert torch.equal(got_x, gx) and torch.equal(got_s, gs), rep


@pytest.mark.parametrize("io", ["f32", "f64"])
@pytest.mark.parametrize("K", [4, 5, 6, 7, 8, 9, 12, 16, 17, 18, 21, 32])
def test_backward_stash_edges(K, io):
    """Recompute with its kept section inputs: below K = 8 the group's
    input and two stashes (LDS and registers with FP32 I/O, registers
    alone with FP64 I/O); from K = 8 also section K/2's input from the
    forward pass, which splits the sections into two halves with stashes
    each (odd K: halves of unequal length); the LDS stash up to K = 17 (the
    largest that fits two workgroups per CU), registers alone above.
    Equal to the saved-output mode to rounding and to the oracle
    adjoint."""
    n = 2 ** 17 + 333
    dt = np.float32 if io == "f32" else np.float64
    sos = W.make_sos(K, 0.5, 0.97, 160 + K)
    x = W.make_signal(n, 161, dt)
    g = W.grad_seed_signal(n, 161, dt)
    rx, rs = run_backward(sos, x, g, adjoint="recompute")
    sx, ss = run_backward(sos, x, g, adjoint="save")
    assert oracle.rel_rms(rx, sx) < 1e-6
    assert row_err(rs, ss) < 1e-10
    ox, os_ = oracle.sosfilt_backward(x.astype(np.float64), sos, g.astype(np.float64))
    assert oracle.rel_rms(rx, ox) < 1e-6
    assert row_err(rs, os_) < 1e-9


@pytest.mark.parametrize("adjoint", ["save", "recompute"])
@pytest.mark.parametrize("io", ["f64", "f32"])
def test_training_step_in_two_calls(io, adjoint):
    """sos_filt_for_backward then sos_filt_backward_stored: y matches the
    oracle at the forward bars, and gx and gsos equal sos_filt_backward's
    bit for bit (the same forward arithmetic fills the workspace)."""
    dt = np.float64 if io == "f64" else np.float32
    n = 2 ** 18 + 77
    sos = W.make_sos(6, 0.5, 0.97, 170)
    p = S.Plan(sos, io_dtype=io, compute_dtype="f64", N=32, adjoint=adjoint)
    x = torch.from_numpy(W.make_signal(n, 171, dt)).to(DEV)
    g = torch.from_numpy(W.grad_seed_signal(n, 171, dt)).to(DEV)
    y, ws = S.filt_for_backward(p, x)
    gx2, gs2 = S.filt_backward_stored(p, x, g, ws)
    gx1, gs1 = S.filt_backward(p, x, g)
    torch.cuda.synchronize()
    assert torch.equal(gx1, gx2) and torch.equal(gs1, gs2)
    ref = oracle.sosfilt(x.cpu().numpy().astype(np.float64), sos)
    assert oracle.rel_rms(y.cpu().numpy(), ref) < (1e-12 if io == "f64" else 1e-6)


@pytest.mark.parametrize("adjoint", ["save", "recompute"])
def test_batched_training_step_in_two_calls(adjoint):
    """The batched pair: y at the channels' samples only (gaps keep their
    value), matching the oracle; gx and gsos equal the one-call batched
    backward bit for bit."""
    lengths = [1, 255, 5000, 70001, 2 ** 17 + 3]
    offsets, pos = [], 0
    for i, n in enumerate(lengths):
        pos = (pos + 3) // 4 * 4 + 1 + i % 3
        offsets.append(pos)
        pos += n + 2
    Ks = [3, 8, 1, 12, 5]
    sos = [W.make_sos(k, 0.5, 0.95, 180 + c) for c, k in enumerate(Ks)]
    plans = [S.Plan(s_, io_dtype="f32", compute_dtype="f64", N=32, adjoint=adjoint) for s_ in sos]
    b = S.Batch(plans, lengths, offsets=offsets)
    xs = [W.make_signal(n, 181 + c, np.float32) for c, n in enumerate(lengths)]
    gs = [W.grad_seed_signal(n, 181 + c, np.float32) for c, n in enumerate(lengths)]
    xb = np.zeros(b.total, np.float32)
    gb = np.zeros(b.total, np.float32)
    for c, o in enumerate(offsets):
        xb[o:o + lengths[c]] = xs[c]
        gb[o:o + lengths[c]] = gs[c]
    xt, gt = torch.from_numpy(xb).to(DEV), torch.from_numpy(gb).to(DEV)
    y0 = torch.full((b.total,), -7.0, dtype=torch.float32, device=DEV)
    y, ws = S.filt_batched_for_backward(b, xt, y0)
    gx2, gs2, _ = S.filt_backward_batched_stored(b, xt, gt, ws)
    gx1, gs1, _ = S.filt_backward_batched(b, xt, gt)
    torch.cuda.synchronize()
    assert torch.equal(gx1, gx2) and torch.equal(gs1, gs2)
    y = y.cpu().numpy()
    mask = np.ones(b.total, bool)
    for c, o in enumerate(offsets):
        n = lengths[c]
        mask[o:o + n] = False
        assert oracle.rel_rms(y[o:o + n], oracle.sosfilt(xs[c].astype(np.float64), sos[c])) < 1e-6, c
    assert np.all(y[mask] == -7.0)



@pytest.mark.parametrize("adjoint", ["save", "recompute"])
def test_batched_training_step_graph_replays_match_eager(adjoint):
    """The batched two-call training step (forward that fills the workspace,
    then the stored adjoint) captured in one HIP graph: with new x and gy
    before each of three replays, y, gx and gsos equal the eager pair's bit
    for bit."""
    import ctypes
    lib = S.lib()
    lengths = [300, 5000, 2 ** 16 + 9]
    Ks = [2, 8, 5]
    sos = [W.make_sos(k, 0.5, 0.95, 190 + c) for c, k in enumerate(Ks)]
    plans = [S.Plan(s_, io_dtype="f32", compute_dtype="f64", N=32, adjoint=adjoint) for s_ in sos]
    b = S.Batch(plans, lengths)
    T = b.total
    x = torch.zeros(T, dtype=torch.float32, device=DEV)
    g = torch.zeros_like(x)
    y, gx = torch.zeros_like(x), torch.zeros_like(x)
    gs = torch.zeros((sum(Ks), 6), dtype=torch.float64, device=DEV)
    ws = torch.empty(max(b.backward_workspace_size(), 16), dtype=torch.uint8, device=DEV)
    vp = ctypes.c_void_p

    def fill(seed):
        x.copy_(torch.from_numpy(W.make_signal(T, seed, np.float32)).to(DEV))
        g.copy_(torch.from_numpy(W.grad_seed_signal(T, seed, np.float32)).to(DEV))

    def step(stream):
        sp = vp(stream.cuda_stream)
        assert lib.sos_filt_batched_for_backward(b.handle, vp(x.data_ptr()), vp(y.data_ptr()),
                                                 vp(ws.data_ptr()), sp) == 0
        assert lib.sos_filt_backward_batched_stored(b.handle, vp(x.data_ptr()), vp(g.data_ptr()),
                                                    vp(gx.data_ptr()), vp(gs.data_ptr()),
                                                    vp(ws.data_ptr()), sp) == 0

    fill(195)
    step(torch.cuda.current_stream())
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=torch.cuda.Stream()):
        step(torch.cuda.current_stream())
    for rep in range(3):
        fill(196 + rep)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = (y.clone(), gx.clone(), gs.clone())
        step(torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert torch.equal(got[0], y) and torch.equal(got[1], gx) and torch.equal(got[2], gs), rep
    # and the eager result is the oracle's on one channel
    o, n = b.offsets[1], lengths[1]
    ref = oracle.sosfilt(x[o:o + n].cpu().numpy().astype(np.float64), sos[1])
    assert oracle.rel_rms(y[o:o + n].cpu().numpy(), ref) < 1e-6

def test_training_step_bad_arguments():
    import ctypes
    lib = S.lib()
    vp = ctypes.c_void_p
    p = S.Plan(W.make_sos(2, 0.5, 0.9, 190), io_dtype="f32")
    n = 4096
    x = torch.zeros(2 * n, dtype=torch.float32, device=DEV)
    ws = torch.empty(lib.sos_backward_workspace_size(p.handle, n), dtype=torch.uint8, device=DEV)
    # y overlapping x, y missing, workspace missing
    assert lib.sos_filt_for_backward(p.handle, vp(x.data_ptr()), vp(x.data_ptr() + 64), n, vp(ws.data_ptr()),
                                     None) == S.SOS_E_ARG
    assert lib.sos_filt_for_backward(p.handle, vp(x.data_ptr()), None, n, vp(ws.data_ptr()), None) == S.SOS_E_ARG
    assert lib.sos_filt_for_backward(p.handle, vp(x.data_ptr()), vp(x.data_ptr() + 4 * n), n, None,
                                     None) == S.SOS_E_ARG
    # n == 0 does nothing and succeeds
    assert lib.sos_filt_for_backward(p.handle, None, None, 0, vp(ws.data_ptr()), None) == S.SOS_OK


@pytest.mark.parametrize("io", ["f64", "f32"])
@pytest.mark.parametrize("adjoint", ["save", "recompute"])
def test_backward_k64(io, adjoint):
    """K = 64, the plan limit, in both modes (the automatic choice keeps
    the outputs here; recompute runs about 1000 forward passes per group
    with its register stash): against the oracle adjoint."""
    dt = np.float64 if io == "f64" else np.float32
    n = 2 ** 14 + 5
    sos = W.make_sos(64, 0.5, 0.9, 195)
    x = W.make_signal(n, 196, dt)
    g = W.grad_seed_signal(n, 196, dt)
    gx, gs = run_backward(sos, x, g, adjoint=adjoint)
    if io == "f64":
        check_f64(x, sos, g, gx, gs, "K=64 %s" % adjoint)
    else:
        rx, rs = oracle.sosfilt_backward(x.astype(np.float64), sos, g.astype(np.float64))
        assert oracle.rel_rms(gx, rx) < 1e-6
        assert row_err(gs, rs) < 1e-9
