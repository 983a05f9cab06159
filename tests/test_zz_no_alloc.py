"""sos_filt_static (the entry point that allocates nothing: the exact carry's
workspace is the library's static device buffer) against sos_filt with a
caller workspace, through the C ABI.

Both run the same kernels in the same order on the same inputs, so their
outputs must be equal bit for bit; both are also held to the FP64 oracle's
bars (FP64 in/out: 1e-12 relative RMS, or four times the oracle's own error
against the extended-precision oracle where that is larger; FP32 in/out:
1e-6).  Each case makes two calls in a row, the second on a shorter signal,
so the second call runs on the buffer the first one left behind.
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


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _with_workspace(plan, xt):
    """sos_filt through the C ABI with a caller-allocated workspace."""
    n = xt.numel()
    ws = plan.workspace_size(n)
    wsb = torch.empty(max(ws, 16), dtype=torch.uint8, device=DEV)
    y = torch.full_like(xt, float("nan"))
    st = S.lib().sos_filt(plan.handle, _ptr(xt), _ptr(y), n, _ptr(wsb), S._stream_ptr(None))
    assert st == S.SOS_OK, S.status_string(st)
    return y


def _static(plan, xt):
    """sos_filt_static through the C ABI."""
    y = torch.full_like(xt, float("nan"))
    st = S.lib().sos_filt_static(plan.handle, _ptr(xt), _ptr(y), xt.numel(), S._stream_ptr(None))
    assert st == S.SOS_OK, S.status_string(st)
    return y


def _check_oracle(y, x_np, sos, io):
    if io == "f32":
        err = oracle.rel_rms(y, oracle.sosfilt(x_np, sos))
        assert err < 1e-6, err
        return
    ld = oracle.sosfilt_ld(x_np, sos)
    err, own = oracle.rel_rms(y, ld), oracle.rel_rms(oracle.sosfilt(x_np, sos), ld)
    assert err <= max(1e-12, 4 * own), (err, own)


@pytest.mark.parametrize("io", ["f64", "f32"])
@pytest.mark.parametrize("K,N", [(8, 16), (16, 64), (3, 8)])
def test_static_equals_workspace_two_calls(io, K, N):
    """Exact carry forced (so the static buffer is used), two calls with the
    second shorter: equal to sos_filt with a workspace, bit for bit."""
    sos = W.make_sos(K, 0.9, 0.999, 700 + K)
    dt = np.float64 if io == "f64" else np.float32
    p = S.Plan(sos, io_dtype=io, compute_dtype="f64", N=N, carry="scan")
    for n, seed in ((2 ** 20 + 5, 701), (2 ** 17 + 3, 702)):
        need = p.workspace_size(n)
        assert 0 < need <= S.SOS_STATIC_SCRATCH_BYTES, need
        x = W.make_signal(n, seed, dt)
        xt = torch.from_numpy(x).to(DEV)
        ys = _static(p, xt)
        yw = _with_workspace(p, xt)
        torch.cuda.synchronize()
        assert torch.equal(ys, yw), (n, float((ys - yw).abs().max()))
        _check_oracle(ys.cpu().numpy(), x, sos, io)


def test_static_run_in_needs_no_buffer():
    """A call that carries by the run-in uses no workspace: same result as
    sos_filt without one."""
    sos = W.make_sos(8, 0.8, 0.98, 0)
    p = S.Plan(sos, io_dtype="f32", compute_dtype="f64", N=64, carry="runin")
    n = 2 ** 20 + 7
    assert p.workspace_size(n) == 0
    x = W.make_signal(n, 703, np.float32)
    xt = torch.from_numpy(x).to(DEV)
    ys = _static(p, xt)
    yw = S.filt(p, xt)
    torch.cuda.synchronize()
    assert torch.equal(ys, yw)
    _check_oracle(ys.cpu().numpy(), x, sos, "f32")


def test_static_rejects_oversize_and_bad_args():
    """More workspace than the static buffer: SOS_E_SCRATCH and y untouched;
    null pointers and n < 0: SOS_E_ARG; n = 0: no-op."""
    sos = W.make_sos(8, 0.9, 0.999, 704)
    # one group per tile makes the tile count, and the carry's buffers, grow
    # with n
    p = S.Plan(sos, io_dtype="f32", compute_dtype="f64", N=8, tile_groups=1, carry="scan")
    n = 2 ** 23
    assert p.workspace_size(n) > S.SOS_STATIC_SCRATCH_BYTES
    xt = torch.zeros(n, dtype=torch.float32, device=DEV)
    y = torch.full_like(xt, 7.0)
    st = S.lib().sos_filt_static(p.handle, _ptr(xt), _ptr(y), n, S._stream_ptr(None))
    assert st == S.SOS_E_SCRATCH
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
    assert S.lib().sos_filt_static(p.handle, None, _ptr(y), n, S._stream_ptr(None)) == S.SOS_E_ARG
    assert S.lib().sos_filt_static(p.handle, _ptr(xt), _ptr(y), -1, S._stream_ptr(None)) == S.SOS_E_ARG
    assert S.lib().sos_filt_static(None, _ptr(xt), _ptr(y), 16, S._stream_ptr(None)) == S.SOS_E_ARG
    assert S.lib().sos_filt_static(p.handle, _ptr(xt), _ptr(y), 0, S._stream_ptr(None)) == S.SOS_OK
    with pytest.raises(S.SosError) as e:
        S.filt_static(p, xt, y)
    assert e.value.code == S.SOS_E_SCRATCH
