"""GPU parity of the exact inter-tile carry (every tile from zero section
states, a log-depth scan of the tile end states, every tile again from its
true state) against the FP64 oracle, and its choice against the run-in.

Tolerances as for the run-in path: FP64 in/out 1e-12 relative RMS, or four
times the FP64 oracle's own error against the extended-precision oracle where
that is larger (poles up to r = 0.999); FP32 in/out 1e-6.
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


def filt(p, x_np):
    y = S.filt(p, torch.from_numpy(x_np).to(DEV))
    torch.cuda.synchronize()
    return y.cpu().numpy()


def check(y, x_np, sos, io):
    if io == "f32":
        err = oracle.rel_rms(y, oracle.sosfilt(x_np, sos))
        assert err < 1e-6, err
        return err
    ld = oracle.sosfilt_ld(x_np.astype(np.float64), sos)
    err, own = oracle.rel_rms(y, ld), oracle.rel_rms(oracle.sosfilt(x_np, sos), ld)
    assert err <= max(1e-12, 4 * own), (err, own)
    return err


@pytest.mark.parametrize("io", ["f64", "f32"])
@pytest.mark.parametrize("N", [16, 64])
@pytest.mark.parametrize("K", [1, 4, 8, 16])
def test_scan_carry_long_run_in(io, N, K):
    """Poles up to r = 0.999 (run-ins of tens of thousands of samples) on a
    signal a few run-ins long: the library takes the scan by itself."""
    sos = W.make_sos(K, 0.9, 0.999, 300 + K)
    dt = np.float64 if io == "f64" else np.float32
    n = 3 * 2 ** 17 + 77
    x = W.make_signal(n, 301, dt)
    p = S.Plan(sos, io_dtype=io, compute_dtype="f64", N=N)
    # the automatic choice: the scan where the run-in exceeds 1.2 tiles and
    # saves at least 8192 section-samples
    w, t = p.info().warm_samples, p.tile(n)
    assert (p.workspace_size(n) > 0) == (5 * w > 6 * t and K * (w - t) >= 8192)
    check(filt(p, x), x, sos, io)
    ps = S.Plan(sos, io_dtype=io, compute_dtype="f64", N=N, carry="scan")
    assert ps.workspace_size(n) > 0
    check(filt(ps, x), x, sos, io)


@pytest.mark.parametrize("n", [1, 1000, 2 ** 16 + 3, 2 ** 20 + 5])
def test_scan_carry_forced_short_run_in(n):
    """Forced on the headline cascade (short run-in): same result as the
    run-in path and the oracle."""
    sos = W.make_sos(8, 0.8, 0.98, 0)
    x = W.make_signal(n, 302, np.float64)
    ps = S.Plan(sos, io_dtype="f64", compute_dtype="f64", N=32, carry="scan")
    pr = S.Plan(sos, io_dtype="f64", compute_dtype="f64", N=32, carry="runin")
    assert ps.workspace_size(n) > 0 and pr.workspace_size(n) == 0
    ys, yr = filt(ps, x), filt(pr, x)
    check(ys, x, sos, "f64")
    check(yr, x, sos, "f64")
    # two FP64 evaluation orders (different tile boundaries); at r <= 0.98
    # FP64 rounding alone puts a direct form 1e-12 off extended precision
    assert oracle.rel_rms(ys, yr) < 1e-11


@pytest.mark.parametrize("offset", [-2, -1, 0, 1])
def test_scan_carry_impulse_across_tiles(offset):
    """A unit impulse next to a tile boundary: the response crosses one or
    more boundaries and matches the oracle's impulse response."""
    sos = W.make_sos(4, 0.95, 0.999, 303)
    p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", N=16, tile_groups=2, carry="scan")
    n = 2 ** 16
    tile = 2 * 16 * 16
    x = np.zeros(n)
    x[3 * tile + offset] = 1.0
    check(filt(p, x), x, sos, "f64")


@pytest.mark.parametrize("solver", ["ph", "cr"])
def test_scan_carry_slow_pole(solver):
    """r = 0.9995, theta = 0.01, close to a double pole at z = 1, on tiles
    of 512 samples: Phi is nearly defective and Phi^512 has entries in the
    hundreds, so its powers and the scan sums lose digits the way PH's
    terminal scan (powers of -C) does at this pole.  The bound is the PH
    family's at this pole (an FP64 model of PH is 6.6e-11 off extended
    precision here)."""
    import math
    r, th = 0.9995, 0.01
    sec = np.array([[1.0, 0.0, 0.0, 1.0, -2 * r * math.cos(th), r * r]])
    x = W.make_signal(2 ** 19, 7, np.float64)
    p = S.Plan(sec, io_dtype="f64", compute_dtype="f64", solver=solver, N=8, tile_groups=4, carry="scan")
    err = oracle.rel_rms(filt(p, x), oracle.sosfilt(x, sec))
    assert err < 2e-10, err


def test_scan_carry_unfactored_b0_and_solvers():
    sos = W.make_sos(3, 0.9, 0.999, 304)
    sos[1, 0] = 0.0                               # b0 = 0: the FIR keeps b0
    x = W.make_signal(2 ** 18 + 9, 305, np.float64)
    for solver in ("ph", "cr", "auto"):
        p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", N=32, solver=solver, carry="scan")
        assert not p.info().b0_factored
        check(filt(p, x), x, sos, "f64")


def test_scan_carry_not_taken_where_unsupported():
    """K > 16, FP32 arithmetic and the comparison solvers keep the run-in:
    no workspace, same results as before."""
    n = 2 ** 17
    assert S.Plan(W.make_sos(17, 0.9, 0.999, 306), io_dtype="f32", carry="scan").workspace_size(n) == 0
    assert S.Plan(W.make_sos(4, 0.9, 0.999, 306), io_dtype="f32", compute_dtype="f32",
                  carry="scan").workspace_size(n) == 0
    assert S.Plan(W.make_sos(4, 0.9, 0.999, 306), io_dtype="f32", solver="scalar",
                  carry="scan").workspace_size(n) == 0
    # the headline workload keeps the run-in
    p = S.Plan(W.make_sos(8, 0.8, 0.98, 0), io_dtype="f32", N=64)
    assert p.workspace_size(2 ** 28) == 0


def test_scan_carry_without_workspace():
    """NULL workspace: the automatic choice falls back to the run-in (same
    result to rounding); a plan that asks for the scan gets SOS_E_ARG."""
    lib = S.lib()
    sos = W.make_sos(8, 0.95, 0.999, 307)
    n = 2 ** 18
    x_np = W.make_signal(n, 308, np.float64)
    x = torch.from_numpy(x_np).to(DEV)
    y = torch.empty_like(x)
    pa = S.Plan(sos, io_dtype="f64", compute_dtype="f64", N=32)
    assert pa.workspace_size(n) > 0
    rc = lib.sos_filt(pa.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), n, None, None)
    assert rc == S.SOS_OK
    torch.cuda.synchronize()
    check(y.cpu().numpy(), x_np, sos, "f64")
    ps = S.Plan(sos, io_dtype="f64", compute_dtype="f64", N=32, carry="scan")
    rc = lib.sos_filt(ps.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), n, None, None)
    assert rc == S.SOS_E_ARG


def test_scan_carry_graph_replays_match_eager():
    """The carry's launches (two tile passes, the powers, the scan rounds)
    captured in a HIP graph with a caller workspace: every replay equals the
    eager call bit for bit."""
    lib = S.lib()
    sos = W.make_sos(6, 0.9, 0.999, 309)
    n = 2 ** 18 + 33
    p = S.Plan(sos, io_dtype="f32", compute_dtype="f64", N=32, carry="scan")
    ws = p.workspace_size(n)
    assert ws > 0
    wsb = torch.empty(ws, dtype=torch.uint8, device=DEV)
    xin = torch.from_numpy(W.make_signal(n, 310, np.float32)).to(DEV)
    yout = torch.empty_like(xin)
    stream = torch.cuda.Stream()

    def call(x, y, s):
        rc = lib.sos_filt(p.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), n,
                          ctypes.c_void_p(wsb.data_ptr()), ctypes.c_void_p(s.cuda_stream))
        assert rc == S.SOS_OK

    call(xin, yout, torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        call(xin, yout, torch.cuda.current_stream())
    for rep in range(3):
        fresh = torch.from_numpy(W.make_signal(n, 311 + rep, np.float32)).to(DEV)
        xin.copy_(fresh)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = yout.clone()
        eager = torch.empty_like(fresh)
        call(fresh, eager, torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert torch.equal(got, eager), rep
