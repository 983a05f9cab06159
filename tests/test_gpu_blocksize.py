"""GPU parity of the block sizes L = 32 and 64 (a group spread over two DPP
rows, or over the whole wavefront) against the FP64 oracle, through the C
ABI.  The method is the same at every L (Section V: L is the block size of
the stride-N layout); only the lane moves differ, so the bars are those of
L = 16: FP64 in/out within 1e-12 relative RMS (or four times the FP64
oracle's own error against its extended-precision twin where that is
larger), FP32 in/out within 1e-6.
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


@pytest.mark.parametrize("L", [32, 64])
@pytest.mark.parametrize("solver", ["ph", "cr"])
def test_tiny_workload_at_its_block_size(solver, L):
    """The small workload as specified (2^16 float64 samples, K = 8,
    r in [0.5, 0.95], N = 8, L = 64) and at L = 32."""
    cfg = W.CONFIGS["tiny"]
    sos = W.make_sos(cfg.K, cfg.r_lo, cfg.r_hi, cfg.seed)
    x = W.make_signal(cfg.n, cfg.seed, np.float64)
    p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", solver=solver, N=8, L=L)
    info = p.info()
    assert info.L == L and info.warm_samples % (8 * L) == 0
    y = filt(p, x)
    assert oracle.rel_rms(y, oracle.sosfilt(x, sos)) < 1e-12


@pytest.mark.parametrize("io", ["f64", "f32"])
@pytest.mark.parametrize("N", [8, 16, 32, 64])
@pytest.mark.parametrize("L", [32, 64])
@pytest.mark.parametrize("solver", ["ph", "cr"])
def test_block_size_every_n(solver, L, N, io):
    """PH and CR at every N, ragged length (a partial last group and tiles
    of several groups), poles up to r = 0.98."""
    sos = W.make_sos(8, 0.8, 0.98, 900 + N + L)
    dt = np.float64 if io == "f64" else np.float32
    n = 3 * 2 ** 16 + 12345
    x = W.make_signal(n, 901, dt)
    p = S.Plan(sos, io_dtype=io, compute_dtype="f64", solver=solver, N=N, L=L)
    check(filt(p, x), x, sos, io, "%s L=%d N=%d %s" % (solver, L, N, io))


@pytest.mark.parametrize("L", [32, 64])
@pytest.mark.parametrize("n", [1, 5, 255, 511, 513, 4097, 70001])
def test_block_size_ragged_lengths(L, n):
    """Lengths shorter than one group, around group and tile boundaries."""
    sos = W.make_sos(3, 0.5, 0.95, 910)
    x = W.make_signal(n, 911, np.float64)
    p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", solver="auto", N=16, L=L, tile_groups=2)
    check(filt(p, x), x, sos, "f64", "n=%d" % n)


@pytest.mark.parametrize("L", [32, 64])
def test_block_size_impulses_across_tiles(L):
    """Unit impulses one sample before and at tile and group boundaries: the
    carry (run-in) and the row-to-row steps inside a wavefront must
    reproduce the oracle's impulse responses across them."""
    sos = W.make_sos(4, 0.9, 0.98, 912)
    N = 16
    p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", solver="ph", N=N, L=L, tile_groups=3)
    n = 40 * N * L + 7
    tile = p.tile(n)
    x = np.zeros(n)
    for pos in (tile - 1, tile, 2 * tile - 1, N * L - 1, 5 * N * L):
        if pos < n:
            x[pos] = 1.0
    check(filt(p, x), x, sos, "f64")


@pytest.mark.parametrize("L", [32, 64])
def test_block_size_cr_guard_and_unfactored_b0(L):
    """The CR hazard angles (routed to PH by the guard) and a section with
    b0 = 0 (b0 kept in the numerator) at L = 32, 64."""
    rows = []
    for th in (np.pi / 2, np.pi / 4, np.pi / 8, np.pi / 2 + 1e-4):
        r = 0.9
        rows.append([0.3, 0.1, 0.2, 1.0, -2 * r * np.cos(th), r * r])
    rows.append([0.0, 0.5, -0.25, 1.0, -0.5, 0.3])
    sos = np.array(rows)
    x = W.make_signal(2 ** 15 + 3, 913, np.float64)
    p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", solver="cr", N=32, L=L)
    assert not p.info().b0_factored
    check(filt(p, x), x, sos, "f64")


def test_block_size_rejected_where_not_built():
    sos = W.make_sos(2, 0.5, 0.9, 914)
    for solver in ("scalar", "block", "phd"):
        with pytest.raises(S.SosError) as e:
            S.Plan(sos, io_dtype="f32", compute_dtype="f64", solver=solver, N=16, L=32)
        assert e.value.code == S.SOS_E_UNSUPPORTED
    for L in (8, 48, 128):
        with pytest.raises(S.SosError) as e:
            S.Plan(sos, io_dtype="f32", compute_dtype="f64", solver="ph", N=16, L=L)
        assert e.value.code == S.SOS_E_UNSUPPORTED
    # the exact carry is built for L = 16: other block sizes carry by the run-in
    p = S.Plan(sos, io_dtype="f64", compute_dtype="f64", solver="ph", N=16, L=64, carry="scan")
    assert p.workspace_size(2 ** 20) == 0


@pytest.mark.parametrize("L", [32, 64])
def test_block_size_batched(L):
    """Ragged channels with their own cascades (K 1..16, PH and CR mixed) in
    one batched launch at L = 32, 64, channels at unaligned offsets with
    gaps; every channel at the single-signal bar, gaps untouched, and a
    graph replay equal to the eager launch."""
    rng = np.random.default_rng(915 + L)
    lengths = [1, 700, 2 ** 14 + 3, 99999, 3 * 2 ** 15]
    offsets, pos = [], 0
    for i, n in enumerate(lengths):
        pos += 1 + i % 3
        offsets.append(pos)
        pos += n
    sos = [W.make_sos(int(rng.integers(1, 17)), 0.5, 0.95, 916 + c) for c in range(len(lengths))]
    plans = [S.Plan(s_, io_dtype="f32", compute_dtype="f64", solver="cr" if c % 2 else "ph", N=16, L=L)
             for c, s_ in enumerate(sos)]
    b = S.Batch(plans, lengths, offsets=offsets)
    xs = [W.make_signal(n, 917 + c, np.float32) for c, n in enumerate(lengths)]
    xb = np.zeros(b.total, np.float32)
    for c, o in enumerate(offsets):
        xb[o:o + lengths[c]] = xs[c]
    xt = torch.from_numpy(xb).to(DEV)
    y0 = torch.full((b.total,), -5.0, dtype=torch.float32, device=DEV)
    y = S.filt_batched(b, xt, y0)
    torch.cuda.synchronize()
    yn = y.cpu().numpy()
    mask = np.ones(b.total, bool)
    for c, o in enumerate(offsets):
        n = lengths[c]
        mask[o:o + n] = False
        check(yn[o:o + n], xs[c], sos[c], "f32", "channel %d" % c)
    assert np.all(yn[mask] == -5.0)
    g = torch.cuda.CUDAGraph()
    yg = torch.full_like(y0, -5.0)
    s = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=s):
        S.filt_batched(b, xt, yg, stream=torch.cuda.current_stream())
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(yg, y)


def test_autotuner_searches_block_size():
    """sos_batch_tune times every (N, L, tile) candidate and reports one of
    them as the fastest; the batch built from it matches the oracle."""
    lengths = [5000, 70001, 2 ** 16]
    sos = [W.make_sos(k, 0.5, 0.95, 920 + k) for k in (2, 8, 5)]
    total = int(sum(lengths))
    x = W.make_signal(total, 921, np.float32)
    xt = torch.from_numpy(x).to(DEV)
    yt = torch.empty_like(xt)
    best, rows = S.batch_tune(sos, lengths, xt, yt, Ns=(16, 32), Ls=(16, 32, 64), tiles=(0, 4), reps=2)
    assert len(rows) == 12 and {r["L"] for r in rows} == {16, 32, 64}
    assert all(r["seconds"] > 0 for r in rows)
    assert best["seconds"] == min(r["seconds"] for r in rows)
    plans = [S.Plan(s_, io_dtype="f32", compute_dtype="f64", solver="ph", N=best["N"], L=best["L"]) for s_ in sos]
    b = S.Batch(plans, lengths, tile_groups=best["tile_groups"])
    y = S.filt_batched(b, xt).cpu().numpy()
    o = 0
    for c, n in enumerate(lengths):
        check(y[o:o + n], x[o:o + n], sos[c], "f32", "channel %d" % c)
        o += n
