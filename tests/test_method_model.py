"""The paper's method, step by step in FP64 (oracle/method.py), against the
definition (the DF1 oracle), the paper's printed worked example, closed forms
of its tables, dense solves and the operation counts of Tables I and III."""
import math
import os
from collections import Counter

import numpy as np
import pytest

import oracle
from oracle import method as M
from paper_2607_14054_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "permutation_L4_N8.txt")


def load_perm_golden():
    stages = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, *blocks = line.split()
        stages[name] = [[int(v) for v in b.split(",")] for b in blocks]
    return stages


def test_permutation_network_matches_printed_example():
    g = load_perm_golden()
    trace = []
    out = M.permutation_network(np.arange(32), N=8, L=4, trace=trace)
    assert [list(map(int, b)) for b in trace[0]] == g["original"]
    assert [list(map(int, b)) for b in trace[1]] == g["regroup"]
    assert [list(map(int, b)) for b in trace[2]] == g["exchange1"]
    assert [list(map(int, b)) for b in out] == g["final"]


@pytest.mark.parametrize("N,L", [(8, 4), (16, 8), (64, 16), (64, 64)])
def test_permutation_network_equals_stride_definition(N, L):
    xg = np.arange(N * L)
    blocks = np.array(M.permutation_network(xg, N, L))
    assert np.array_equal(blocks, M.strided_blocks(xg, N, L))
    assert np.array_equal(M.unstrided(M.strided_blocks(xg, N, L)), xg)


def test_u_tables_closed_form_and_zero_input_response():
    a1, a2 = -1.3, 0.8
    u1, u2 = M.u_tables(a1, a2, 40)
    # the first entries printed in Section VI-A
    assert (u2[0], u1[0]) == (a2, a1)
    assert u2[1] == -a1 * a2 and u1[1] == a2 - a1 * a1
    # u_{1,m} = -(zero-input response to y[-1] = 1); u_{2,m} likewise for y[-2]
    sec = np.array([[1.0, 0.0, 0.0, 1.0, a1, a2]])
    z = np.zeros(40)
    r1 = oracle.sosfilt(z, sec, zi=[[0, 0, 0, 1.0]])
    r2 = oracle.sosfilt(z, sec, zi=[[0, 0, 1.0, 0]])
    assert np.allclose(u1, -r1, rtol=0, atol=1e-14)
    assert np.allclose(u2, -r2, rtol=0, atol=1e-14)


@pytest.mark.parametrize("N", [4, 8, 64])
def test_C_is_minus_state_transition_power(N):
    a1, a2 = 0.9, 0.6
    T = np.array([[0.0, 1.0], [-a2, -a1]])   # (y[n-2], y[n-1]) -> (y[n-1], y[n])
    assert np.allclose(M.ph_C(a1, a2, N), -np.linalg.matrix_power(T, N), atol=1e-15)


def test_sklansky_equals_sequential_recurrence():
    rng = np.random.default_rng(0)
    C = rng.standard_normal((2, 2)) * 0.4
    we = rng.standard_normal((64, 2))
    ops = Counter()
    ys = M.sklansky_2x2(we, C, ops)
    ref = we.copy()
    for l in range(1, 64):
        ref[l] = we[l] - C @ ref[l - 1]
    assert np.allclose(ys, ref, atol=1e-12)
    assert ops["rd_fma"] == 2 * 6 and ops["rd_shuffle"] == 4 * 6 + 1


@pytest.mark.parametrize("r,theta", [(0.9, 0.3), (0.97, 2.2), (0.5, 1.1)])
def test_cr_coefficients_closed_form(r, theta):
    a1, a2 = -2 * r * math.cos(theta), r * r
    rows, (eT, fT) = M.cr_coefficients(a1, a2, 6)
    for i, (c, d, fe, e, f) in enumerate(rows):
        # the reduced polynomial has the squared roots: pole pair r^(2^i) e^(+-j 2^i theta)
        assert math.isclose(e, -2 * r ** (2 ** i) * math.cos(2 ** i * theta), rel_tol=1e-12, abs_tol=1e-15)
        assert math.isclose(f, r ** (2 ** (i + 1)), rel_tol=1e-12)
        assert math.isclose(c, e - f / e, rel_tol=1e-12) and math.isclose(d, -f * f / e, rel_tol=1e-12)
    assert math.isclose(eT, -2 * r ** 64 * math.cos(64 * theta), rel_tol=1e-9, abs_tol=1e-15)
    assert math.isclose(fT, r ** 128, rel_tol=1e-9)


def test_permuted_system_dense_solve_with_state():
    """eq. recursive_equation_multi_block_form with explicit matrices and a
    nonzero initial state equals the definition."""
    rng = np.random.default_rng(1)
    N, L = 8, 4
    b1, b2, a1, a2 = 0.3, -0.2, -1.1, 0.7
    x = rng.standard_normal(N * L)
    xs, ys = rng.standard_normal(2), rng.standard_normal(2)
    A, Am = M.dense_multiblock(a1, a2, N, L)
    B, Bm = M.dense_multiblock(b1, b2, N, L)
    xg = M.strided_blocks(x, N, L).reshape(-1)
    yg = np.linalg.solve(A, B @ xg + Bm @ xs - Am @ ys)
    sec = np.array([[1.0, b1, b2, 1.0, a1, a2]])
    ref = oracle.sosfilt(x, sec, zi=[[xs[0], xs[1], ys[0], ys[1]]])
    assert np.allclose(M.unstrided(yg.reshape(N, L)), ref, atol=1e-13)
    # the non-recursive stage of eq. feedforward_block_uniform gives the same rhs
    V = M.nonrecursive_stage(M.strided_blocks(x, N, L), 1.0, b1, b2, a1, a2, xs, ys)
    assert np.allclose(V.reshape(-1), B @ xg + Bm @ xs - Am @ ys, atol=1e-14)


@pytest.mark.parametrize("solver", ["ph", "cr"])
@pytest.mark.parametrize("N,L", [(4, 16), (8, 64), (16, 8), (64, 4), (2, 32)])
def test_method_equals_definition(solver, N, L):
    sos = W.make_sos(8, 0.5, 0.95, 0)
    x = W.make_signal(N * L * 5 + 77, 1)      # ragged tail
    y = oracle.sosfilt(x, sos)
    assert oracle.rel_rms(M.filter_groups(x, sos, N, L, solver), y) < 2e-12


def test_cr_terminal_forms_agree():
    rng = np.random.default_rng(2)
    V = rng.standard_normal((16, 32))
    a = M.cr_solve(V, -0.9, 0.5, terminal="block")
    b = M.cr_solve(V, -0.9, 0.5, terminal="sequential")
    assert np.allclose(a, b, atol=1e-13)


@pytest.mark.parametrize("N,L", [(8, 8), (64, 8), (16, 64)])
def test_operation_counts_match_tables(N, L):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((N, L))
    lg = int(math.log2(L))
    ops = Counter()
    V = M.nonrecursive_stage(X, 1.0, 0.1, 0.2, -0.5, 0.3, (0, 0), (0, 0), ops)
    M.ph_solve(V, -0.5, 0.3, ops)
    ph = ops["nonrec_fma"] + ops["particular_fma"] + ops["rd_fma"] + ops["homog_fma"]
    assert ph == 6 * N + 2 * lg - 4                         # Table I total
    sh = ops["nonrec_shuffle"] + ops["rd_shuffle"] + ops["homog_shuffle"]
    assert sh == 4 * lg + 5
    ops = Counter()
    V = M.nonrecursive_stage(X, 1.0, 0.1, 0.2, -0.5, 0.3, (0, 0), (0, 0), ops)
    M.cr_solve(V, -0.5, 0.3, ops)
    cr = ops["nonrec_fma"] + ops["reduction_fma"] + ops["terminal_fma"] + ops["backsub_fma"]
    assert cr == 6 * N + L - 1                              # Table III total
    lgN = int(math.log2(N))
    assert ops["reduction_fma"] == 2 * N - 2 and ops["backsub_fma"] == 2 * N - 2
    assert ops["reduction_shuffle"] == lgN and ops["backsub_shuffle"] == lgN + 1



@pytest.mark.parametrize("N,L", [(64, 16), (8, 16), (32, 64)])
def test_bench_flop_count_is_the_models(N, L):
    """The FP64 roofline that bench.py reports prices each section at the
    FMAs per sample that the method model counts per group (Tables I, III)."""
    import bench
    X = np.random.default_rng(4).standard_normal((N, L))
    per = {}
    for solver, solve, keys in (("ph", M.ph_solve, ("particular_fma", "rd_fma", "homog_fma")),
                                ("cr", M.cr_solve, ("reduction_fma", "terminal_fma", "backsub_fma"))):
        ops = Counter()
        V = M.nonrecursive_stage(X, 1.0, 0.1, 0.2, -0.5, 0.3, (0, 0), (0, 0), ops)
        solve(V, -0.5, 0.3, ops)
        per[solver] = (ops["nonrec_fma"] + sum(ops[k] for k in keys)) / N
    got = bench.algorithmic_fma_per_sample(["ph", "cr", "ph"], N, L)
    assert got == pytest.approx(2 * per["ph"] + per["cr"], rel=1e-15)

def test_method_in_float32_is_near_plain_float32():
    """The FP32 accuracy floor: the method in float32 lands at the level of a
    plain float32 sequential cascade on the same draw (both far from FP64)."""
    sos = W.make_sos(8, 0.5, 0.95, 0)
    x = W.make_signal(8192, 0, np.float32)
    y = oracle.sosfilt(x, sos)
    plain = oracle.rel_rms(oracle.sosfilt_f32arith(x, sos), y)
    ph = oracle.rel_rms(M.filter_groups(x, sos, 8, 64, "ph", dtype=np.float32), y)
    assert ph < 10 * plain + 1e-6
