"""GPU parity of the comparison solvers against the FP64 oracle: scalar
filtering (SOS_SCALAR) and block filtering (SOS_BLOCK) with FP64, FP16 and
BF16 Toeplitz products.

Tolerances (relative RMS against the FP64 oracle):
* FP64 arithmetic and FP64 I/O: 1e-12 on r <= 0.95 draws; for the K = 16
  draw, within max(1e-12, 4x) of the FP64 oracle's own error against the
  long-double oracle.
* FP32 I/O with FP64 arithmetic: 1e-6.
* FP16 / BF16 products (FP32 accumulation, FP64 carries): these are a
  precision study.  The bounds below are stated results for these draws,
  about 4x above what was measured, not a parity bar.
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


def run(sos, x_np, **kw):
    io = "f64" if x_np.dtype == np.float64 else "f32"
    p = S.Plan(sos, io_dtype=io, **kw)
    y = S.filt(p, torch.from_numpy(x_np).to(DEV))
    torch.cuda.synchronize()
    return y.cpu().numpy(), p


@pytest.mark.parametrize("solver", ["scalar", "block"])
@pytest.mark.parametrize("K", [1, 5, 8, 16])
def test_variant_f64_tiny_config(solver, K):
    sos = W.make_sos(K, 0.5, 0.95, 60 + K)
    x = W.make_signal(2 ** 16, 61, np.float64)
    y, _ = run(sos, x, compute_dtype="f64", solver=solver)
    # arbitrated by the long-double oracle: deep cascades attenuate so much
    # that the FP64 oracle's own error approaches 1e-12
    ld = oracle.sosfilt_ld(x, sos)
    err, own = oracle.rel_rms(y, ld), oracle.rel_rms(oracle.sosfilt(x, sos), ld)
    print("%s K=%d rel_rms=%.2e (oracle %.2e)" % (solver, K, err, own))
    assert err <= max(1e-12, 4 * own)


@pytest.mark.parametrize("solver", ["scalar", "block"])
@pytest.mark.parametrize("n", [1, 3, 31, 33, 255, 257, 4097, 100003])
def test_variant_ragged(solver, n):
    sos = W.make_sos(4, 0.5, 0.95, 62)
    x = W.make_signal(n, 63, np.float64)
    y, _ = run(sos, x, compute_dtype="f64", solver=solver, tile_groups=2)
    assert oracle.rel_rms(y, oracle.sosfilt(x, sos)) < 1e-12


@pytest.mark.parametrize("solver,unit", [("scalar", 32), ("block", 256)])
@pytest.mark.parametrize("offset", [-2, -1, 0, 1])
def test_variant_impulse_across_tile_boundary(solver, unit, offset):
    sos = W.make_sos(8, 0.5, 0.95, 64)
    tg = 3
    tile = unit * tg
    n = 40 * tile
    x = np.zeros(n)
    x[7 * tile + offset] = 1.0
    y, _ = run(sos, x, compute_dtype="f64", solver=solver, tile_groups=tg)
    ref = oracle.sosfilt(x, sos)
    assert np.max(np.abs(y - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("solver", ["scalar", "block"])
def test_variant_f32_io(solver):
    sos = W.make_sos(8, 0.8, 0.98, 0)
    x = W.make_signal(2 ** 20 + 777, 0, np.float32)
    y, _ = run(sos, x, compute_dtype="f64", solver=solver)
    err = oracle.rel_rms(y, oracle.sosfilt(x, sos))
    print("%s f32 io rel_rms=%.2e" % (solver, err))
    assert err < 1e-6


def test_scalar_unfactored_b0():
    sos = W.make_sos(3, 0.5, 0.95, 65)
    sos[1, 0:3] = [0.0, 0.4, 0.3]
    x = W.make_signal(30000, 66, np.float64)
    y, p = run(sos, x, compute_dtype="f64", solver="scalar")
    assert not p.info().b0_factored
    assert oracle.rel_rms(y, oracle.sosfilt(x, sos)) < 1e-12


# measured rel_rms on these draws, times about four (precision study)
LOW_PRECISION_BOUND = {("f16", 0.95): 2e-2, ("bf16", 0.95): 1e-1}


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_block_low_precision_products(dtype):
    """FP16 / BF16 Toeplitz products with FP32 accumulation and FP64 carries,
    K = 8, r in [0.5, 0.95]: finite, and within the stated error."""
    sos = W.make_sos(8, 0.5, 0.95, 67)
    x = W.make_signal(2 ** 18, 68, np.float32)
    y, p = run(sos, x, compute_dtype=dtype, solver="block")
    assert p.info().compute_dtype == dtype
    ref = oracle.sosfilt(x, sos)
    err = oracle.rel_rms(y, ref)
    print("block %s rel_rms=%.3e max_rel=%.3e" % (dtype, err, oracle.max_rel(y, ref)))
    assert np.all(np.isfinite(y))
    assert err < LOW_PRECISION_BOUND[(dtype, 0.95)]


def test_low_precision_only_with_block():
    sos = W.make_sos(2, 0.5, 0.9, 69)
    for dt in ("f16", "bf16"):
        with pytest.raises(S.SosError) as e:
            S.Plan(sos, io_dtype="f32", compute_dtype=dt, solver="ph")
        assert e.value.code == S.SOS_E_UNSUPPORTED
    with pytest.raises(S.SosError) as e:
        S.Plan(W.make_sos(17, 0.5, 0.9, 69), io_dtype="f32", solver="scalar")
    assert e.value.code == S.SOS_E_UNSUPPORTED
