"""GPU parity of wide groups, N = 128 .. 1024 blocks per lane run (the upper
half of the paper's N sweep), against the FP64 oracle through the C ABI.
N = 128 with FP32 I/O keeps a lane's run in registers (a wavefront alone
on its SIMD); the other wide plans keep the runs in the caller's workspace,
all-PH plans with one pass over it per section, the deferred-correction PH
(AUTO's choice there) with one pass for all sections.  PH, cyclic reduction
(log2 N = 7 .. 10 levels) and the deferred PH.  Bars as for N <= 64: FP64
in/out within 1e-12 relative RMS (or four times the FP64 oracle's own error
against its extended-precision twin where that is larger), FP32 in/out
within 1e-6.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2607_14054_amd import sosfilt as S
from paper_2607_14054_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
WIDE_N = [128, 256, 512, 1024]


def filt(p, x_np):
    y = S.filt(p, torch.from_numpy(x_np).to(DEV))
    torch.cuda.synchronize()
    return y.cpu().numpy()


def check(y, x, sos, io, what=""):
    if io == "f32":
        err = oracle.rel_rms(y, oracle.sosfilt(x, sos))
        assert err < 1e-6, (what, err)
        return err
    ld = oracle.sosfilt_ld(x.astype(np.float64), sos)
    err, own = oracle.rel_rms(y, ld), oracle.rel_rms(oracle.sosfilt(x, sos), ld)
    assert err <= max(1e-12, 4 * own), (what, err, own)
    return err


@pytest.mark.parametrize("io", ["f64", "f32"])
@pytest.mark.parametrize("N", WIDE_N)
@pytest.mark.parametrize("solver", ["ph", "cr", "auto"])
def test_wide_groups(solver, N, io):
    """K = 8, r in [0.8, 0.98], several groups per tile plus a ragged tail
    (AUTO is the deferred PH where the runs live in the workspace, PH in
    registers)."""
    sos = W.make_sos(8, 0.8, 0.98, 930 + N)
    dt = np.float64 if io == "f64" else np.float32
    n = 9 * 16 * N + 4321
    x = W.make_signal(n, 931, dt)
    p = S.Plan(sos, io_dtype=io, compute_dtype="f64", solver=solver, N=N, tile_groups=2)
    info = p.info()
    if solver == "auto":
        assert info.solver == ["phd" if (N > 128 or io == "f64") else "ph"] * 8
    # N = 128 with FP32 I/O keeps its lane runs in registers, the other wide
    # plans keep them in the workspace
    assert info.N == N and (p.workspace_size(n) > 0) == (N > 128 or io == "f64")
    check(filt(p, x), x, sos, io, "%s N=%d %s" % (solver, N, io))


@pytest.mark.parametrize("N", WIDE_N)
def test_wide_tiny_and_ragged(N):
    """Lengths below one group and around group boundaries, K = 1 and 3."""
    for K, n in ((1, 1), (3, 17), (3, 16 * N - 1), (1, 16 * N + 1), (3, 3 * 16 * N + 5)):
        sos = W.make_sos(K, 0.5, 0.95, 932 + K)
        x = W.make_signal(n, 933, np.float64)
        p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", solver="auto", N=N, tile_groups=1)
        check(filt(p, x), x, sos, "f64", "N=%d K=%d n=%d" % (N, K, n))


@pytest.mark.parametrize("solver", ["ph", "cr"])
def test_wide_impulses_across_tiles(solver):
    """Impulses one sample before and at group and tile boundaries, N = 256."""
    N = 256
    sos = W.make_sos(4, 0.9, 0.98, 934)
    p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", solver=solver, N=N, tile_groups=2)
    n = 7 * 16 * N + 11
    tile = p.tile(n)
    x = np.zeros(n)
    for pos in (16 * N - 1, 16 * N, tile - 1, tile, 2 * tile - 1, N - 1, N):
        x[pos] = 1.0
    check(filt(p, x), x, sos, "f64")


def test_wide_cr_guard_routes_to_ph():
    """The CR hazard angles at N = 1024 (ten levels): the guard sends those
    sections to PH, the rest run CR, and the result is the oracle's."""
    rows = []
    for th in (np.pi / 2, np.pi / 4, np.pi / 8, 1.0, 2.0):
        r = 0.9
        rows.append([0.3, 0.1, 0.2, 1.0, -2 * r * np.cos(th), r * r])
    sos = np.array(rows)
    p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", solver="cr", N=1024)
    assert "ph" in p.info().solver and "cr" in p.info().solver
    x = W.make_signal(5 * 16 * 1024 + 3, 935, np.float64)
    check(filt(p, x), x, sos, "f64")


def test_wide_needs_its_workspace():
    """N > 64 without a workspace (or a misaligned one): SOS_E_ARG and no
    launch; the static-scratch entry point refuses the size."""
    p = S.Plan(W.make_sos(2, 0.5, 0.9, 936), io_dtype="f32", compute_dtype="f64", N=512)
    n = 2 ** 24   # 2048 groups, 512 wavefronts of 256 KB
    assert p.workspace_size(n) > S.SOS_STATIC_SCRATCH_BYTES
    x = torch.zeros(n, dtype=torch.float32, device=DEV)
    y = torch.full_like(x, 3.0)
    vp = ctypes.c_void_p
    assert S.lib().sos_filt(p.handle, vp(x.data_ptr()), vp(y.data_ptr()), n, None,
                            S._stream_ptr(None)) == S.SOS_E_ARG
    assert S.lib().sos_filt_static(p.handle, vp(x.data_ptr()), vp(y.data_ptr()), n,
                                   S._stream_ptr(None)) == S.SOS_E_SCRATCH
    torch.cuda.synchronize()
    assert bool((y == 3.0).all())


@pytest.mark.parametrize("solver", ["ph", "phd"])
@pytest.mark.parametrize("N", [256, 1024])
def test_wide_static_scratch_matches(N, solver):
    """sos_filt_static on a wide plan whose workspace fits the static
    buffer gives sos_filt's output bit for bit, twice in a row (the second
    call shorter)."""
    sos = W.make_sos(8, 0.8, 0.98, 939)
    p = S.Plan(sos, io_dtype="f32", compute_dtype="f64", solver=solver, N=N)
    for n in (9 * 16 * N + 77, 3 * 16 * N + 5):
        assert 0 < p.workspace_size(n) <= S.SOS_STATIC_SCRATCH_BYTES
        x = torch.from_numpy(W.make_signal(n, 940 + n % 7, np.float32)).to(DEV)
        want = S.filt(p, x)
        got = torch.full_like(x, 7.0)
        S.filt_static(p, x, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), n


@pytest.mark.parametrize("n", [1, 17, 16 * 256 - 1, 16 * 256 + 1, 5 * 16 * 256 + 3, 70001])
def test_wide_ph_one_pass_ragged(n):
    """The all-PH wide kernel (one pass over the run per section) and AUTO's
    deferred PH (one pass for all sections) at N = 256, FP32 I/O: lengths
    below one group and around group boundaries, K = 3 and a b0 = 0 section
    (b0 kept in the numerator)."""
    sos = W.make_sos(3, 0.5, 0.95, 937)
    for b0zero in (False, True):
        s_ = sos.copy()
        if b0zero:
            s_[1, 0:3] = [0.0, 0.5, -0.25]
        x = W.make_signal(n, 938, np.float32)
        for solver in ("ph", "auto"):
            p = S.Plan(s_, io_dtype="f32", compute_dtype="f64", solver=solver, N=256, tile_groups=2)
            assert p.workspace_size(n) > 0 and p.info().b0_factored == (not b0zero)
            check(filt(p, x), x, s_, "f32", "%s n=%d b0zero=%s" % (solver, n, b0zero))


@pytest.mark.parametrize("solver", ["ph", "cr"])
@pytest.mark.parametrize("N", [128, 256, 1024])
def test_wide_headline_full_size_sampled(N, solver):
    """The full headline workload (2^28 float32 samples, K = 8, r in
    [0.8, 0.98], seed 0) at N = 128 and 1024 in the launch shape the bench
    sweep times, on windows at the start, across tile boundaries, in the
    middle and at the end (each against the oracle run from four run-ins
    before it)."""
    c = W.CONFIGS["scale"]
    sos = W.make_sos(c.K, c.r_lo, c.r_hi, c.seed)
    x_np = W.make_signal(c.n, c.seed, np.float32)
    p = S.Plan(sos, io_dtype="f32", compute_dtype="f64", solver=solver, N=N)
    tile, W_run = p.tile(c.n), p.info().warm_samples
    x = torch.from_numpy(x_np).to(DEV)
    y = S.filt(p, x)
    torch.cuda.synchronize()
    for start in (0, tile - 7, 100 * tile - 3, c.n // 2 + 123, c.n - 3000):
        lo = max(0, start - 4 * W_run)
        hi = min(start + 3000, c.n)
        ref = oracle.sosfilt(x_np[lo:hi], sos)[start - lo:]
        err = oracle.rel_rms(y[start:hi].cpu().numpy(), ref)
        assert err < 1e-6, (N, solver, start, err)


@pytest.mark.parametrize("N,solver", [(4, "cr"), (128, "auto"), (256, "ph"), (512, "cr")])
def test_wide_and_narrow_graph_replays(N, solver):
    """sos_filt captured in a HIP graph (workspace allocated beforehand)
    replays equal to the eager launch, three times with new inputs in
    between."""
    sos = W.make_sos(6, 0.8, 0.98, 941)
    p = S.Plan(sos, io_dtype="f32", compute_dtype="f64", solver=solver, N=N)
    n = 7 * 16 * N + 333
    ws = p.workspace_size(n)
    wsb = torch.empty(max(ws, 16), dtype=torch.uint8, device=DEV)
    x = torch.from_numpy(W.make_signal(n, 942, np.float32)).to(DEV)
    y = torch.empty_like(x)
    vp = ctypes.c_void_p

    def launch(stream_ptr):
        rc = S.lib().sos_filt(p.handle, vp(x.data_ptr()), vp(y.data_ptr()), n,
                              vp(wsb.data_ptr()) if ws else None, stream_ptr)
        assert rc == S.SOS_OK, rc

    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    launch(S._stream_ptr(None))
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        launch(S._stream_ptr(s))
    for rep in range(3):
        x.copy_(torch.from_numpy(W.make_signal(n, 943 + rep, np.float32)).to(DEV))
        y.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        got = y.clone()
        launch(S._stream_ptr(None))
        torch.cuda.synchronize()
        assert torch.equal(got, y), (N, rep)
        check(y.cpu().numpy(), x.cpu().numpy(), sos, "f32", "N=%d rep %d" % (N, rep))


@pytest.mark.parametrize("io", ["f64", "f32"])
@pytest.mark.parametrize("K", [1, 3, 8, 13, 16])
@pytest.mark.parametrize("N", WIDE_N)
def test_wide_deferred(N, K, io):
    """The deferred-correction PH on wide groups (all sections zero-state in
    one pass over the run, the corrections of every section at the end on
    MFMA): K = 1 .. 16 (the three register classes of its zero-state
    histories), several groups per tile and a ragged tail."""
    sos = W.make_sos(K, 0.8, 0.98, 950 + K)
    dt = np.float64 if io == "f64" else np.float32
    n = 9 * 16 * N + 4321
    x = W.make_signal(n, 951, dt)
    p = S.Plan(sos, io_dtype=io, compute_dtype="f64", solver="phd", N=N, tile_groups=2)
    assert p.info().N == N and set(p.info().solver) == {"phd"}
    assert p.workspace_size(n) > 0
    check(filt(p, x), x, sos, io, "phd N=%d K=%d %s" % (N, K, io))


@pytest.mark.parametrize("N", [128, 1024])
def test_wide_deferred_tiny_ragged_and_impulses(N):
    """Lengths below one group and around group and tile boundaries, and
    impulses just before and at them (K = 5)."""
    sos = W.make_sos(5, 0.9, 0.98, 952)
    p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", solver="phd", N=N, tile_groups=1)
    for n in (1, 17, 16 * N - 1, 16 * N + 1, 3 * 16 * N + 5):
        x = W.make_signal(n, 953, np.float64)
        check(filt(p, x), x, sos, "f64", "N=%d n=%d" % (N, n))
    n = 6 * 16 * N + 7
    x = np.zeros(n)
    for pos in (N - 1, N, 16 * N - 1, 16 * N, 2 * 16 * N - 2):
        x[pos] = 1.0
    check(filt(p, x), x, sos, "f64", "impulses N=%d" % N)


def test_wide_deferred_full_size_sampled():
    """The full headline workload (2^28 float32 samples, K = 8) by the
    deferred PH at N = 512 in the launch shape the bench sweep times, on
    windows at the start, across a tile boundary, in the middle and at the
    end."""
    c = W.CONFIGS["scale"]
    sos = W.make_sos(c.K, c.r_lo, c.r_hi, c.seed)
    x_np = W.make_signal(c.n, c.seed, np.float32)
    p = S.Plan(sos, io_dtype="f32", compute_dtype="f64", solver="phd", N=512)
    tile, W_run = p.tile(c.n), p.info().warm_samples
    x = torch.from_numpy(x_np).to(DEV)
    y = S.filt(p, x)
    torch.cuda.synchronize()
    for start in (0, tile - 7, c.n // 2 + 123, c.n - 3000):
        lo = max(0, start - 4 * W_run)
        hi = min(start + 3000, c.n)
        ref = oracle.sosfilt(x_np[lo:hi], sos)[start - lo:]
        err = oracle.rel_rms(y[start:hi].cpu().numpy(), ref)
        assert err < 1e-6, (start, err)
