"""Host side of the C ABI, no GPU: symbol exports, argument validation, and the
FP64 plan tables against closed forms and against the FP64 method model."""
import math
import os
import re

import numpy as np
import pytest

import oracle
from oracle import method as M
from paper_2607_14054_amd import sosfilt as S
from paper_2607_14054_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "sosfilt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const char\s*\*|sos_status|size_t|int64_t)\s*\*?\s*(sos_\w+)\s*\(",
                                 text, re.M)))


def test_library_exports_every_declared_symbol():
    import ctypes
    names = header_functions()
    assert len(names) >= 7
    lib = S.lib()
    for n in names:
        assert hasattr(lib, n), n
        assert ctypes.cast(getattr(lib, n), ctypes.c_void_p).value
    assert set(S.EXPORTED) <= set(names)


def plan(sos, **kw):
    kw.setdefault("host_only", True)
    return S.Plan(sos, **kw)


def test_status_strings():
    assert S.status_string(S.SOS_OK) == "ok"
    assert "coefficient" in S.status_string(S.SOS_E_COEF)


@pytest.mark.parametrize("bad,code", [
    ("a0", S.SOS_E_COEF), ("nan", S.SOS_E_COEF), ("inf", S.SOS_E_COEF),
    ("unstable_a2", S.SOS_E_UNSTABLE), ("unstable_a1", S.SOS_E_UNSTABLE),
])
def test_coefficient_validation(bad, code):
    sos = W.make_sos(3, 0.5, 0.9, 1)
    if bad == "a0":
        sos[1, 3] = 0.0
    elif bad == "nan":
        sos[2, 1] = np.nan
    elif bad == "inf":
        sos[0, 5] = np.inf
    elif bad == "unstable_a2":
        sos[1, 5] = 1.0
    elif bad == "unstable_a1":
        sos[1, 4], sos[1, 5] = -1.6, 0.5
    with pytest.raises(S.SosError) as e:
        plan(sos)
    assert e.value.code == code


@pytest.mark.parametrize("kw,code", [
    (dict(N=2), S.SOS_E_UNSUPPORTED), (dict(N=24), S.SOS_E_UNSUPPORTED),
    # narrow groups (N = 4): 16-lane rows, PH or CR only
    (dict(N=4, L=32), S.SOS_E_UNSUPPORTED), (dict(N=4, solver="scalar"), S.SOS_E_UNSUPPORTED),
    (dict(N=4, solver="phd"), S.SOS_E_UNSUPPORTED),
    (dict(N=2048), S.SOS_E_UNSUPPORTED), (dict(io_dtype="f64", compute_dtype="f32"), S.SOS_E_UNSUPPORTED),
    # wide groups (N > 64): FP64 arithmetic, 16-lane rows, PH, CR or the
    # deferred-correction PH only
    (dict(N=128, compute_dtype="f32"), S.SOS_E_UNSUPPORTED), (dict(N=256, L=32), S.SOS_E_UNSUPPORTED),
    (dict(N=512, solver="scalar"), S.SOS_E_UNSUPPORTED), (dict(N=1024, solver="block"), S.SOS_E_UNSUPPORTED),
])
def test_option_validation(kw, code):
    with pytest.raises(S.SosError) as e:
        plan(W.make_sos(2, 0.5, 0.9, 1), **kw)
    assert e.value.code == code


def test_empty_cascade_rejected():
    with pytest.raises((S.SosError, ValueError)):
        plan(np.zeros((0, 6)))


def test_rows_normalised_and_b0_factored():
    sos = W.make_sos(4, 0.5, 0.9, 2)
    sos[2] *= 2.5                                  # a0 = 2.5
    p = plan(sos, compute_dtype="f64")
    info = p.info()
    assert info.b0_factored
    rows, gain = M.normalise(sos)
    for k in range(4):
        assert np.allclose(p.table(S.SOS_TABLE_ROWS, k), rows[k], rtol=1e-15, atol=0)
    assert math.isclose(info.gain, gain, rel_tol=1e-14)


def test_b0_zero_keeps_unfactored_rows():
    sos = W.make_sos(3, 0.5, 0.9, 3)
    sos[1, 0:3] = [0.0, 1.0, 0.5]
    p = plan(sos)
    assert not p.info().b0_factored and p.info().gain == 1.0
    assert np.allclose(p.table(S.SOS_TABLE_ROWS, 1), [0.0, 1.0, 0.5, sos[1, 4], sos[1, 5]])


@pytest.mark.parametrize("N", [4, 8, 16, 32, 64])
def test_ph_tables_match_model(N):
    sos = W.make_sos(3, 0.6, 0.97, 4)
    p = plan(sos, N=N, solver="ph")
    rows, _ = M.normalise(sos)
    for k in range(3):
        a1, a2 = rows[k, 3], rows[k, 4]
        u1, u2 = M.u_tables(a1, a2, N)
        assert np.allclose(p.table(S.SOS_TABLE_U1, k), u1, rtol=1e-13, atol=1e-300)
        assert np.allclose(p.table(S.SOS_TABLE_U2, k), u2, rtol=1e-13, atol=1e-300)
        C = M.ph_C(a1, a2, N)
        assert np.allclose(p.table(S.SOS_TABLE_C, k).reshape(2, 2), C, rtol=1e-13, atol=1e-300)
        pw = p.table(S.SOS_TABLE_PH_POWERS, k).reshape(4, 2, 2)    # L = 16: log2 L rounds
        for j in range(4):
            assert np.allclose(pw[j], np.linalg.matrix_power(-C, 2 ** j), rtol=1e-10, atol=1e-300)
    assert p.info().solver == ["ph"] * 3


@pytest.mark.parametrize("N", [4, 8, 16, 64])
def test_cr_tables_match_closed_form(N):
    r, theta = 0.93, 0.7
    sec = np.array([[1.0, 0.1, 0.2, 1.0, -2 * r * math.cos(theta), r * r]])
    p = plan(sec, N=N, solver="cr")
    lv = p.table(S.SOS_TABLE_CR_LEVELS, 0).reshape(-1, 4)
    lg = int(math.log2(N))
    assert lv.shape == (lg, 4)
    for i in range(lg):
        e = -2 * r ** (2 ** i) * math.cos(2 ** i * theta)
        f = r ** (2 ** (i + 1))
        fe, ee, c, d = lv[i]
        assert math.isclose(ee, e, rel_tol=1e-11, abs_tol=1e-15)
        assert math.isclose(fe, f / e, rel_tol=1e-10)
        assert math.isclose(c, e - f / e, rel_tol=1e-10) and math.isclose(d, -f * f / e, rel_tol=1e-10)
    eT, fT = p.table(S.SOS_TABLE_CR_TERMINAL, 0)
    assert math.isclose(eT, -2 * r ** N * math.cos(N * theta), rel_tol=1e-8, abs_tol=1e-15)
    assert math.isclose(fT, r ** (2 * N), rel_tol=1e-8)
    T = np.array([[0.0, 1.0], [-fT, -eT]])
    pw = p.table(S.SOS_TABLE_CR_POWERS, 0).reshape(4, 2, 2)
    for j in range(4):
        assert np.allclose(pw[j], np.linalg.matrix_power(T, 2 ** j), rtol=1e-10, atol=1e-300)
    assert p.info().solver == ["cr"]


@pytest.mark.parametrize("theta,N", [(math.pi / 2, 8), (math.pi / 4, 8), (math.pi / 8, 64)])
def test_cr_guard_falls_back_to_ph(theta, N):
    """e^(i) = -2 r^(2^i) cos(2^i theta) vanishes at these angles."""
    r = 0.9
    sec = np.array([[1.0, 0.0, 0.0, 1.0, -2 * r * math.cos(theta), r * r]])
    assert plan(sec, N=N, solver="cr").info().solver == ["ph"]
    # auto takes PH whatever the guard says
    assert plan(sec, N=N, solver="auto", compute_dtype="f32").info().solver == ["ph"]


def test_auto_takes_ph():
    """AUTO is PH where the runs stay on chip (N <= 64, and N = 128 with
    FP32 I/O in registers) and the deferred-correction PH where they live in
    the workspace (N = 256 .. 1024, N = 128 with FP64 I/O) up to K = 16;
    PH above K = 16."""
    sos = W.make_sos(8, 0.8, 0.98, 0)
    for N in (4, 8, 16, 32, 64, 128, 256, 1024):
        for io in ("f32", "f64"):
            wide_ws = N > 128 or (N == 128 and io == "f64")
            want = "phd" if wide_ws else "ph"
            assert plan(sos, N=N, io_dtype=io).info().solver == [want] * 8, (N, io)
        assert plan(sos, N=N, solver="cr").info().solver == ["cr"] * 8
        assert plan(sos, N=N, solver="ph").info().solver == ["ph"] * 8
    big = W.make_sos(17, 0.8, 0.98, 0)
    assert plan(big, N=512).info().solver == ["ph"] * 17


def test_cr_flush_of_negligible_levels():
    r = 0.05
    sec = np.array([[1.0, 0.0, 0.0, 1.0, -2 * r * math.cos(1.0), r * r]])
    p = plan(sec, N=64, solver="cr")
    lv = p.table(S.SOS_TABLE_CR_LEVELS, 0).reshape(-1, 4)
    # r^(2^i) < 2^-60 from i = 5 on (0.05^32 ~ 2e-42)
    assert np.all(lv[5:] == 0.0) and np.all(lv[:3] != 0.0)
    assert list(p.table(S.SOS_TABLE_CR_TERMINAL, 0)) == [0.0, 0.0]
    assert p.info().solver == ["cr"]


def test_transition_matches_oracle_one_step():
    """One column of the transition = the oracle's state after one zero input
    sample, starting from a unit state (scaled domain, b0 factored)."""
    sos = W.make_sos(3, 0.5, 0.95, 5)
    p = plan(sos)
    rows, _ = M.normalise(sos)
    K = 3
    Phi = p.table(S.SOS_TABLE_TRANSITION).reshape(2 * K, 2 * K)
    scaled = np.column_stack([rows[:, 0:3], np.ones(K), rows[:, 3:5]])
    for col in range(2 * K):
        s = np.zeros(2 * K); s[col] = 1.0
        zi = np.zeros((K, 4))
        for k in range(K):
            zi[k, 2:4] = s[2 * k:2 * k + 2]
            if k > 0:
                zi[k, 0:2] = s[2 * (k - 1):2 * k]
        _, zf = oracle.sosfilt(np.zeros(1), scaled, zi=zi, return_zf=True)
        assert np.allclose(Phi[:, col], zf[:, 2:4].reshape(-1), atol=1e-15)


def test_run_in_length_bounds_transition():
    sos = W.make_sos(8, 0.8, 0.98, 0)
    p = plan(sos, N=32)
    info = p.info()
    K = 8
    Phi = p.table(S.SOS_TABLE_TRANSITION).reshape(2 * K, 2 * K)
    P = np.linalg.matrix_power(Phi, info.warm_samples)
    # 2^16 below FP32's unit roundoff, the precision of the stored outputs
    assert np.max(np.sum(np.abs(P), axis=1)) < 2.0 ** -40
    assert info.warm_samples % (32 * 16) == 0
    assert math.isclose(info.transition_norm_W, np.max(np.sum(np.abs(P), axis=1)), rel_tol=1e-6)
    # the run-in is not absurdly long: the slowest pole is 0.98
    assert info.warm_samples <= 16 * 2048


@pytest.mark.parametrize("io,eps", [("f32", 2.0 ** -40), ("f64", 2.0 ** -64)])
@pytest.mark.parametrize("draw", [(8, 0.8, 0.98, 0), (4, 0.5, 0.95, 7), (2, 0.9, 0.99, 3)])
def test_run_in_is_the_shortest_whole_group_length_below_its_bound(io, eps, draw):
    """W is the first multiple of N L at which the transition's infinity
    norm falls below the bound of the stored type (2^-40 for FP32 output,
    2^16 below its unit roundoff; 2^-64 for FP64): one group less does not
    reach it.  The transition is the plan's table, which
    test_transition_matches_oracle_one_step pins to the oracle."""
    sos = W.make_sos(*draw)
    N, L = 32, 16
    p = plan(sos, N=N, io_dtype=io, compute_dtype="f64")
    info = p.info()
    K = sos.shape[0]
    Phi = p.table(S.SOS_TABLE_TRANSITION).reshape(2 * K, 2 * K)
    def norm(w):
        return np.max(np.sum(np.abs(np.linalg.matrix_power(Phi, w)), axis=1))
    G = N * L
    W_run = info.warm_samples
    assert W_run % G == 0 and W_run >= G
    assert norm(W_run) < eps
    assert W_run == G or norm(W_run - G) >= eps


def test_run_in_truncation_is_negligible_in_the_oracle():
    """Starting a tile from zero state W samples early changes it far below
    FP32's rounding of the outputs (the truncation is below 2^-40)."""
    sos = W.make_sos(8, 0.8, 0.98, 0)
    info = plan(sos, N=8).info()
    x = W.make_signal(info.warm_samples + 5000, 0)
    full = oracle.sosfilt(x, sos)[info.warm_samples:]
    # the truncated run starts from zero at sample 0 of a longer signal
    pre = np.concatenate([np.random.default_rng(1).standard_normal(20000), x])
    late = oracle.sosfilt(pre, sos)[20000 + info.warm_samples:]
    assert oracle.rel_rms(late, full) < 1e-10


@pytest.mark.parametrize("N", [16, 32, 256])
def test_deferred_tables_match_oracle_responses(N):
    """Theta and the coupling blocks of the deferred correction are the
    cascade's responses to unit entry states, computed here by the oracle
    (scaled rows: b0 factored, as the kernels use them)."""
    K = 3
    sos = W.make_sos(K, 0.5, 0.95, 41)
    p = plan(sos, N=N, solver="phd")
    assert p.info().solver == ["phd"] * K
    rows, _ = M.normalise(sos)
    scaled = np.column_stack([rows[:, 0:3], np.ones(K), rows[:, 3:5]])
    Theta = p.table(S.SOS_TABLE_THETA).reshape(N, 2 * K)
    for j in range(K):
        for c in range(2):
            zi = np.zeros((K, 4))
            zi[j, 2 + c] = 1.0                  # y_j history
            if j + 1 < K:
                zi[j + 1, c] = 1.0              # x_{j+1} = y_j history
            out = oracle.sosfilt(np.zeros(N), scaled, zi=zi)
            assert np.allclose(Theta[:, 2 * j + c], out, rtol=1e-12, atol=1e-14)
            for k in range(j + 1, K):
                part = oracle.sosfilt(np.zeros(N), scaled[:k + 1], zi=zi[:k + 1])
                blk = p.table(S.SOS_TABLE_COUPLING, k).reshape(k, 2, 2)[j]
                assert np.allclose(blk[:, c], part[N - 2:N], rtol=1e-12, atol=1e-14)
    # the diagonal blocks are -C of the PH factorisation
    for k in range(K):
        C = p.table(S.SOS_TABLE_C, k).reshape(2, 2)
        zi = np.zeros((K, 4))
        resp = np.zeros((2, 2))
        for c in range(2):
            zi[:] = 0.0
            zi[k, 2 + c] = 1.0
            out = oracle.sosfilt(np.zeros(N), scaled[k:k + 1], zi=zi[k:k + 1])
            resp[:, c] = out[N - 2:N]
        assert np.allclose(resp, -C, rtol=1e-12, atol=1e-15)


def test_deferred_solver_limits():
    sos = W.make_sos(4, 0.5, 0.9, 1)
    for kw in (dict(N=8), dict(compute_dtype="f32", N=32)):
        with pytest.raises(S.SosError) as e:
            plan(sos, solver="phd", **kw)
        assert e.value.code == S.SOS_E_UNSUPPORTED
    with pytest.raises(S.SosError):
        plan(W.make_sos(17, 0.5, 0.9, 1), solver="phd", N=16)
    # wide groups: up to K = 16 too
    assert plan(W.make_sos(16, 0.5, 0.9, 1), solver="phd", N=1024).info().solver == ["phd"] * 16
    with pytest.raises(S.SosError):
        plan(W.make_sos(17, 0.5, 0.9, 1), solver="phd", N=256)
    # auto takes cyclic reduction with the guard's PH fallback
    assert set(plan(sos, N=32).info().solver) <= {"cr", "ph"}
    assert set(plan(W.make_sos(17, 0.5, 0.9, 1), N=16).info().solver) <= {"cr", "ph"}


# ---------------------------------------------------------------- batches

def _host_plans(Ks, N=32, io="f32", seed=0):
    return [S.Plan(W.make_sos(int(k), 0.5, 0.95, seed + c), io_dtype=io, N=N, host_only=True)
            for c, k in enumerate(Ks)]


@pytest.mark.parametrize("cap", [0, 1, 3, 32])
def test_batch_schedule_covers_every_channel(cap):
    rng = np.random.default_rng(7)
    C = 40
    lengths = np.floor(2.0 ** rng.uniform(0, 20, size=C)).astype(np.int64)
    lengths[[3, 17]] = 0
    Ks = rng.integers(1, 17, size=C)
    N = 16
    G = N * 16
    b = S.Batch(_host_plans(Ks, N=N), lengths, tile_groups=cap, host_only=True)
    q = b.query()
    # dense packing in channel order
    assert np.array_equal(q["offsets"], np.concatenate([[0], np.cumsum(lengths)[:-1]]))
    assert q["total"] == lengths.sum()
    assert sorted(q["order"].tolist()) == list(range(C))
    items = 0
    for c in range(C):
        t = int(q["tile"][c])
        assert t > 0 and t % G == 0
        if cap:
            assert t <= cap * G
        # the tiles cover [-shift, n): shift = samples past the last 16-byte
        # boundary before the channel start (4 float32 samples per 16 bytes)
        span = int(lengths[c]) + int(q["offsets"][c]) % 4 if lengths[c] else 0
        ntiles = -(-span // t)
        quads = -(-ntiles // 4)
        # tiles as even as the length allows: the quads could not be fewer
        if ntiles:
            assert (quads - 1) * 4 * t < span + 4 * t
        items += quads
    assert q["items"] == items


def test_batch_order_costliest_first():
    Ks = [1, 16, 4]
    lengths = [2 ** 20, 2 ** 20, 2 ** 20]
    b = S.Batch(_host_plans(Ks), lengths, host_only=True)
    assert b.query()["order"].tolist() == [1, 2, 0]


def test_batch_explicit_offsets():
    b = S.Batch(_host_plans([2, 3, 4]), [100, 0, 50], offsets=[1000, 5, 0], host_only=True)
    q = b.query()
    assert q["offsets"].tolist() == [1000, 5, 0] and q["total"] == 1100
    with pytest.raises(S.SosError) as e:
        S.Batch(_host_plans([2, 3]), [100, 100], offsets=[0, 99], host_only=True)
    assert e.value.code == S.SOS_E_ARG
    with pytest.raises(S.SosError) as e:
        S.Batch(_host_plans([2]), [10], offsets=[-1], host_only=True)
    assert e.value.code == S.SOS_E_ARG


def test_batch_rejections():
    mixed_n = _host_plans([2], N=16) + _host_plans([2], N=32)
    with pytest.raises(S.SosError) as e:
        S.Batch(mixed_n, [10, 10], host_only=True)
    assert e.value.code == S.SOS_E_UNSUPPORTED
    mixed_io = _host_plans([2], io="f32") + _host_plans([2], io="f64")
    with pytest.raises(S.SosError) as e:
        S.Batch(mixed_io, [10, 10], host_only=True)
    assert e.value.code == S.SOS_E_UNSUPPORTED
    block_ph = [S.Plan(W.make_sos(2, 0.5, 0.9, 0), N=32, solver=s_, host_only=True) for s_ in ("block", "ph")]
    with pytest.raises(S.SosError) as e:
        S.Batch(block_ph, [10, 10], host_only=True)
    assert e.value.code == S.SOS_E_UNSUPPORTED
    blocks = S.Batch(block_ph[:1] * 3, [10, 700, 70000], host_only=True)
    assert blocks.query()["total"] == 70710
    phd = [S.Plan(W.make_sos(2, 0.5, 0.9, 0), N=32, solver="phd", host_only=True)]
    with pytest.raises(S.SosError) as e:
        S.Batch(phd, [10], host_only=True)
    assert e.value.code == S.SOS_E_UNSUPPORTED
    with pytest.raises(S.SosError) as e:
        S.Batch(_host_plans([2]), [-1], host_only=True)
    assert e.value.code == S.SOS_E_ARG
    # host-only plans cannot back a device batch; a host-only batch cannot filter
    with pytest.raises(S.SosError) as e:
        S.Batch(_host_plans([2]), [10])
    assert e.value.code == S.SOS_E_ARG
    import ctypes
    b = S.Batch(_host_plans([2]), [10], host_only=True)
    assert S.lib().sos_filt_batched(b.handle, None, None, None, None) == S.SOS_E_ARG
    assert S.lib().sos_batch_plan(None, 1, None, None, None, None) == S.SOS_E_ARG


def test_batch_replan_host_only():
    b = S.Batch(_host_plans([2, 3, 4]), [100, 2000, 50], host_only=True)
    assert b.query()["total"] == 2150
    b.replan(_host_plans([5, 1, 8, 2, 16]), [10, 0, 70000, 3, 12345])
    q = b.query()
    assert b.C == 5 and q["total"] == 10 + 70000 + 3 + 12345
    assert sorted(q["order"].tolist()) == list(range(5))
    # an invalid request leaves the batch as it was
    with pytest.raises(S.SosError) as e:
        b.replan(_host_plans([2], N=16) + _host_plans([2], N=32), [10, 10])
    assert e.value.code == S.SOS_E_UNSUPPORTED
    with pytest.raises(S.SosError) as e:
        b.replan(_host_plans([2, 2]), [10, 10], offsets=[0, 5])
    assert e.value.code == S.SOS_E_ARG
    assert b.query()["total"] == q["total"]


def test_carry_flags():
    """The carry flags: either one is accepted, both together or an unknown
    flag is SOS_E_ARG; a host-only plan has no exact carry (no workspace)."""
    import ctypes
    sos = np.ascontiguousarray(W.make_sos(2, 0.5, 0.9, 1))
    ptr = sos.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def rc(flags):
        h = ctypes.c_void_p()
        o = S._Opts(S.SOS_F32, S.SOS_F64, S.SOS_AUTO, 32, 16, 0, S.SOS_FLAG_HOST_ONLY | flags)
        r = S.lib().sos_plan(ptr, 2, ctypes.byref(o), ctypes.byref(h))
        if r == S.SOS_OK:
            S.lib().sos_plan_destroy(h)
        return r

    assert rc(S.SOS_FLAG_CARRY_SCAN) == S.SOS_OK
    assert rc(S.SOS_FLAG_CARRY_RUNIN) == S.SOS_OK
    assert rc(S.SOS_FLAG_CARRY_SCAN | S.SOS_FLAG_CARRY_RUNIN) == S.SOS_E_ARG
    assert rc(0x40) == S.SOS_E_ARG
    p = S.Plan(W.make_sos(4, 0.9, 0.999, 1), host_only=True, carry="scan")
    assert p.workspace_size(1 << 20) == 0


@pytest.mark.parametrize("N", [128, 256, 512, 1024])
def test_wide_plan_tables(N):
    """Wide groups build the same tables at their N: u closed forms up to
    N, CR levels up to log2 N = 10 (the guard and flush included)."""
    sos = W.make_sos(3, 0.5, 0.95, 7)
    p = plan(sos, N=N, solver="cr")
    assert p.info().N == N
    assert p.table(S.SOS_TABLE_U1, 0).shape == (N,)
    assert p.table(S.SOS_TABLE_CR_LEVELS, 0).shape == (4 * int(np.log2(N)),)


def test_wide_launch_keeps_runs_in_cache():
    """Wide plans on 2^28 samples: one wavefront per SIMD (1024); PH and CR,
    which pass the runs once per section, are capped so that the runs of
    all wavefronts (N x 64 doubles each) fit the 256 MB last-level cache
    (512 wavefronts at N = 1024); the deferred PH is not."""
    n = 2 ** 28
    sos = W.make_sos(8, 0.8, 0.98, 0)

    def waves(p):
        return -(-(-(-n // p.tile(n))) // 4)

    for N, want in ((256, 1024), (512, 1024), (1024, 512)):
        for solver in ("ph", "cr"):
            got = waves(plan(sos, N=N, solver=solver))
            assert got == want, (N, solver, got)
            assert got * N * 64 * 8 <= 256 << 20
        assert waves(plan(sos, N=N, solver="phd")) == 1024
