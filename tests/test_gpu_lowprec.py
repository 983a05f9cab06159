"""GPU parity of block filtering with FP16 / BF16 Toeplitz products against
the FP64 oracle, element by element, under the a-priori error bound of
tests/lowprec_bound.py (derived from the product types' unit roundoffs and
the slicing, never from the kernel's output), for every slice count.

With the default slice counts (3 for FP16, 4 for BF16) two targets hold as
well: on the precision workload's channels the error is at most that of a
plain FP32 sequential cascade on the same channel (the FP32 floor, from the
oracle's FP32 twin), and on the headline cascade's draw it is within 1e-4
relative RMS.
"""
import numpy as np
import pytest

import oracle
from paper_2607_14054_amd import sosfilt as S
from paper_2607_14054_amd import workloads as W

import lowprec_bound as LB

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
DEFAULT_SLICES = {"f16": 3, "bf16": 4}


def check_bounds(y, x, sos, dtype, slices, what):
    """y (the kernel's output) against oracle.sosfilt: every sample within the
    elementwise bound, and the whole signal within the l2 bound; returns the
    relative RMS error."""
    ref = oracle.sosfilt(x, sos)
    B, L2 = LB.error_bounds(x, sos, dtype, slices)
    allow = LB.output_allowance(ref, x, sos)
    d = np.abs(np.asarray(y, dtype=np.float64) - ref)
    assert np.all(np.isfinite(y)), what
    ratio = float(np.max(d / (B + allow)))
    l2 = float(np.linalg.norm(d))
    l2_bound = L2 + float(np.linalg.norm(allow))
    err = oracle.rel_rms(y, ref)
    print("%s %s S=%d: rel_rms %.3e, l2 %.3e of bound %.3e, max |err| / elementwise bound %.3e"
          % (what, dtype, slices, err, l2, l2_bound, ratio))
    assert ratio <= 1.0, (what, ratio)
    assert l2 <= l2_bound, (what, l2, l2_bound)
    return err


@pytest.mark.parametrize("slices", [1, 2, 3, 4])
@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_block_lowprec_within_a_priori_bound(dtype, slices):
    """K = 8, r in [0.5, 0.95], 2^17 float32 samples, one launch."""
    sos = W.make_sos(8, 0.5, 0.95, 67)
    x = W.make_signal(2 ** 17, 68, np.float32)
    p = S.Plan(sos, io_dtype="f32", compute_dtype=dtype, solver="block", slices=slices)
    assert p.info().block_slices == slices
    y = S.filt(p, torch.from_numpy(x).to(DEV))
    torch.cuda.synchronize()
    check_bounds(y.cpu().numpy(), x, sos, dtype, slices, "r<=0.95")


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_block_lowprec_each_slice_adds_its_bits(dtype):
    """Each slice adds W bits (10 for FP16, 8 for BF16) to both operands:
    from one slice count to the next the error falls by at least 2^(W-4),
    until it reaches the FP32 output's own rounding (K = 8, r in [0.5,
    0.95])."""
    W_bits = LB.SLICE_BITS[dtype]
    sos = W.make_sos(8, 0.5, 0.95, 67)
    x = W.make_signal(2 ** 17, 68, np.float32)
    ref = oracle.sosfilt(x, sos)
    out_floor = oracle.rel_rms(ref.astype(np.float32), ref)
    errs = []
    for slices in (1, 2, 3, 4):
        p = S.Plan(sos, io_dtype="f32", compute_dtype=dtype, solver="block", slices=slices)
        y = S.filt(p, torch.from_numpy(x).to(DEV))
        torch.cuda.synchronize()
        errs.append(oracle.rel_rms(y.cpu().numpy(), ref))
    print("%s errors by slices: %s (output rounding %.2e)" % (dtype, errs, out_floor))
    for a, b in zip(errs, errs[1:]):
        assert b <= max(a / 2 ** (W_bits - 4), 4 * out_floor), errs


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_block_lowprec_default_slices(dtype):
    p = S.Plan(W.make_sos(2, 0.5, 0.9, 1), io_dtype="f32", compute_dtype=dtype, solver="block")
    assert p.info().block_slices == DEFAULT_SLICES[dtype]
    with pytest.raises(S.SosError) as e:
        S.Plan(W.make_sos(2, 0.5, 0.9, 1), io_dtype="f32", compute_dtype="f64", solver="block", slices=2)
    assert e.value.code == S.SOS_E_UNSUPPORTED
    with pytest.raises(S.SosError) as e:
        S.Plan(W.make_sos(2, 0.5, 0.9, 1), io_dtype="f32", compute_dtype=dtype, solver="block", slices=5)
    assert e.value.code == S.SOS_E_ARG


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_block_lowprec_precision_workload(dtype):
    """The precision workload at its full size, in the launch the benchmark
    times (256 channels x 2^20 float32 samples, K = 8, r in [0.9, 0.999],
    one batched launch, default slices): sampled channels within the bound
    and at or below the FP32 floor."""
    cfg = W.CONFIGS["precision"]
    C, n = cfg.channels, cfg.n
    sos = [W.make_sos(cfg.K, cfg.r_lo, cfg.r_hi, cfg.seed + c) for c in range(C)]
    xb = torch.empty(C * n, dtype=torch.float32, device=DEV)
    for c in range(C):
        xb[c * n:(c + 1) * n] = torch.from_numpy(W.make_signal(n, cfg.seed + c, np.float32)).to(DEV)
    plans = [S.Plan(s_, io_dtype="f32", compute_dtype=dtype, solver="block", N=64) for s_ in sos]
    b = S.Batch(plans, [n] * C)
    y = S.filt_batched(b, xb)
    torch.cuda.synchronize()
    for c in (0, 1, C // 3, C // 2, C - 1):
        x_c = xb[c * n:(c + 1) * n].cpu().numpy()
        err = check_bounds(y[c * n:(c + 1) * n].cpu().numpy(), x_c, sos[c], dtype, DEFAULT_SLICES[dtype],
                           "precision channel %d" % c)
        floor = oracle.rel_rms(oracle.sosfilt_f32arith(x_c, sos[c]), oracle.sosfilt(x_c, sos[c]))
        assert err <= floor, (c, err, floor)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_block_lowprec_headline_draw(dtype):
    """The headline cascade (K = 8, r in [0.8, 0.98], seed 0) on the first
    2^20 samples of its signal, default slices: within the bound and within
    1e-4 relative RMS of the FP64 oracle (a plain FP32 cascade is 1.3e-3
    off on this draw)."""
    sos = W.make_sos(8, 0.8, 0.98, 0)
    x = W.make_signal(2 ** 20, 0, np.float32)
    p = S.Plan(sos, io_dtype="f32", compute_dtype=dtype, solver="block")
    y = S.filt(p, torch.from_numpy(x).to(DEV))
    torch.cuda.synchronize()
    err = check_bounds(y.cpu().numpy(), x, sos, dtype, DEFAULT_SLICES[dtype], "headline draw")
    assert err <= 1e-4, err
