"""FP64 model of the paper's multi-block method (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product.
It shares no code with the HIP path.

``oracle.sosfilt`` is the plain definition of what the path computes.  This
module instead takes the method's own steps, in the paper's order and
notation, so that each step can be checked against the definition and so
that the plan tables the library computes can be compared with tables built
here from the paper's recurrences.  Notation:

* group of N*L samples, block m (m = 0..N-1) is the stride-N block
  xbar_m[l] = x[m + l N] (Section V, after eq. recursive_equation_multi_block_form);
* R is the lower shift (R v)[0] = 0, (R v)[l] = v[l-1] (Section V, eq. multi_block_A);
* the non-recursive stage is eq. feedforward_block_uniform;
* PH: particular solution (eq. particular_recurrence), terminal 2x2 scan
  (eq. recursive_doubling_equation, realised by Sklansky doubling), and the
  homogeneous correction (eq. PH_forward) with the u tables of Section VI-A;
* CR: log2 N reduction levels with the coefficient update of eq.
  cr_coeff_update, the terminal block of eq. cr_terminal_block solved by
  block filtering (eq. block_filtering_equation) and back substitution
  (eqs. cr_companion_block, cr_backsub_penultimate, cr_backsub_final);
* the cascade keeps the permuted layout between sections (Section VII-B).

Every array here is float64 unless a dtype is passed to ``filter_groups``
(used only to estimate what the same steps give in float32).
"""
from __future__ import annotations

import math
from collections import Counter

import numpy as np


# --------------------------------------------------------------------------
# layout: Section V (strided blocks) and Section VII-A (permutation network)
# --------------------------------------------------------------------------

def strided_blocks(xg: np.ndarray, N: int, L: int) -> np.ndarray:
    """X[m, l] = x[m + l N]: the definition of the stride-N blocks."""
    assert xg.shape[0] == N * L
    return np.ascontiguousarray(xg.reshape(L, N).T)


def unstrided(X: np.ndarray) -> np.ndarray:
    """Inverse of ``strided_blocks``."""
    return np.ascontiguousarray(X.T).reshape(-1)


def permutation_network(xg: np.ndarray, N: int, L: int, trace: list | None = None):
    """The two-phase block permutation of Section VII-A.

    Phase 1 regroups: the N contiguous blocks are split into N/L groups of L
    blocks, group g holding blocks g, g + N/L, g + 2N/L, ...  Phase 2 applies
    log2 L levels of anti-diagonal quadrant exchange inside every L x L
    sub-matrix (columns = blocks, rows = elements), halving the sub-matrix
    each level.  Requires N to be a multiple of L.  Returns the N blocks.
    """
    assert N % L == 0 and (L & (L - 1)) == 0
    blocks = [xg[i * L:(i + 1) * L].copy() for i in range(N)]
    if trace is not None:
        trace.append([b.copy() for b in blocks])
    G = N // L
    regrouped = [blocks[g + G * j] for g in range(G) for j in range(L)]
    if trace is not None:
        trace.append([b.copy() for b in regrouped])
    out = [b.copy() for b in regrouped]
    size = L
    while size > 1:
        h = size // 2
        for g in range(G):
            base = g * L
            for q0 in range(0, L, size):           # sub-matrices along columns
                for c in range(h):
                    left = out[base + q0 + c]
                    right = out[base + q0 + h + c]
                    for r0 in range(0, L, size):   # and along rows
                        lo = slice(r0 + h, r0 + size)   # lower-left quadrant rows
                        up = slice(r0, r0 + h)          # upper-right quadrant rows
                        tmp = left[lo].copy()
                        left[lo] = right[up]
                        right[up] = tmp
        size = h
        if trace is not None:
            trace.append([b.copy() for b in out])
    return out


def R(v: np.ndarray, times: int = 1) -> np.ndarray:
    """Lower shift applied ``times`` times (zeros enter at element 0)."""
    out = v
    for _ in range(times):
        s = np.zeros_like(out)
        s[1:] = out[:-1]
        out = s
    return out


# --------------------------------------------------------------------------
# tables (Section VI)
# --------------------------------------------------------------------------

def u_tables(a1: float, a2: float, N: int):
    """u_{1,m}, u_{2,m} for m = 0..N-1 (Section VI-A, after eq. U_12)."""
    u1 = np.zeros(N)
    u2 = np.zeros(N)
    u2[0], u1[0] = a2, a1
    if N > 1:
        u2[1], u1[1] = -a1 * a2, a2 - a1 * a1
    for m in range(2, N):
        u1[m] = -a2 * u1[m - 2] - a1 * u1[m - 1]
        u2[m] = -a2 * u2[m - 2] - a1 * u2[m - 1]
    return u1, u2


def ph_C(a1: float, a2: float, N: int) -> np.ndarray:
    """C = [[e, g], [f, d]] of eq. C with e, g, f, d from eq. H_22."""
    u1, u2 = u_tables(a1, a2, N)
    return np.array([[u2[N - 2], u1[N - 2]], [u2[N - 1], u1[N - 1]]])


def cr_coefficients(a1: float, a2: float, levels: int):
    """Per level i: (c, d, f/e, e, f) from eq. cr_coeff_update, and the final
    (e, f) of the terminal block (eq. cr_terminal_block)."""
    e, f = a1, a2
    rows = []
    for _ in range(levels):
        rows.append((e - f / e, -f * f / e, f / e, e, f))
        e, f = 2 * f - e * e, f * f
    return rows, (e, f)


def toeplitz_impulse(e: float, f: float, L: int) -> np.ndarray:
    """First L taps of 1 / (1 + e z^-1 + f z^-2): the dense lower-triangular
    Toeplitz inverse used by block filtering (Section IV, eq.
    block_filtering_matrices)."""
    h = np.zeros(L)
    h[0] = 1.0
    if L > 1:
        h[1] = -e
    for j in range(2, L):
        h[j] = -e * h[j - 1] - f * h[j - 2]
    return h


# --------------------------------------------------------------------------
# one section on one group
# --------------------------------------------------------------------------

def nonrecursive_stage(X, b0, b1, b2, a1, a2, xs, ys, ops: Counter | None = None):
    """v = B x + B_- x_-1 - A_- y_-1 via eq. feedforward_block_uniform.

    xs = (x[-2], x[-1]), ys = (y[-2], y[-1]) of this section from the
    preceding group.  b0 multiplies the current block (b0 = 1 in the
    normalised form of eq. simple_second_order).
    """
    N, L = X.shape
    xm1 = R(X[N - 1]); xm1[0] = xs[1]         # extended block xbar_{-1}
    xm2 = R(X[N - 2]); xm2[0] = xs[0]         # extended block xbar_{-2}
    ext = lambda m: X[m] if m >= 0 else (xm1 if m == -1 else xm2)
    V = np.empty_like(X)
    for m in range(N):
        V[m] = b0 * X[m] + b1 * ext(m - 1) + b2 * ext(m - 2)
    V[0][0] -= a1 * ys[1] + a2 * ys[0]
    V[1][0] -= a2 * ys[1]
    if ops is not None:
        ops["nonrec_fma"] += 2 * N + 3
        ops["nonrec_shuffle"] += 2
    return V


def sklansky_2x2(we: np.ndarray, C: np.ndarray, ops: Counter | None = None):
    """Solve ye[l] = we[l] - C ye[l-1], ye[0] = we[0] (eq.
    recursive_doubling_equation) by Sklansky doubling: in the level with span
    2^j, every element of the upper half of each 2^(j+1)-block adds the
    matching power of -C times the last element of the lower half."""
    L = we.shape[0]
    y = we.copy()
    A = -C
    pw = [np.eye(2)]
    for _ in range(L):
        pw.append(A @ pw[-1])
    span = 1
    while span < L:
        for start in range(0, L, 2 * span):
            last = start + span - 1
            for i in range(last + 1, min(start + 2 * span, L)):
                y[i] = y[i] + pw[i - last] @ y[last]
        span *= 2
        if ops is not None:
            ops["rd_fma"] += 2
    if ops is not None:
        ops["rd_shuffle"] += 4 * int(math.log2(L)) + 1
    return y


def ph_solve(V, a1, a2, ops: Counter | None = None):
    """Recursive stage by PH factorisation (Section VI-B, steps 1-3)."""
    N, L = V.shape
    W = np.empty_like(V)
    for m in range(N):                           # step 1, eq. particular_recurrence
        w = V[m].copy()
        if m >= 1:
            w = w - a1 * W[m - 1]
        if m >= 2:
            w = w - a2 * W[m - 2]
        W[m] = w
    if ops is not None:
        ops["particular_fma"] += 2 * N - 3
    C = ph_C(a1, a2, N)                          # step 2, terminal blocks
    we = np.stack([W[N - 2], W[N - 1]], axis=1)  # we[l] = (w[(l+1)N-2], w[(l+1)N-1])
    ye = sklansky_2x2(we, C, ops)
    Y = np.empty_like(V)
    Y[N - 2], Y[N - 1] = ye[:, 0], ye[:, 1]
    u1, u2 = u_tables(a1, a2, N)                 # step 3, eq. PH_forward
    p, q = R(Y[N - 2]), R(Y[N - 1])
    for m in range(N - 2):
        Y[m] = W[m] - u2[m] * p - u1[m] * q
    if ops is not None:
        ops["homog_fma"] += 2 * (N - 2)
        ops["homog_shuffle"] += 2
    return Y


def _wrapped(blocks, idx, p):
    """Block at level position p, wrapping modulo the level size with one R
    per wrap (Section VI-C: indices below zero wrap and the coupling becomes
    the shift R)."""
    n = len(idx)
    w = 0
    while p < 0:
        p += n
        w += 1
    return R(blocks[idx[p]], w)


def cr_solve(V, a1, a2, ops: Counter | None = None, terminal: str = "block"):
    """Recursive stage by cyclic reduction (Section VI-C)."""
    N, L = V.shape
    levels = int(math.log2(N))
    assert 1 << levels == N
    rows, (eT, fT) = cr_coefficients(a1, a2, levels)
    Vp = V.copy()
    for i in range(levels):                      # reduction
        s = 1 << i
        idx = [s * (j + 1) - 1 for j in range(N // s)]
        c, d, fe, e, f = rows[i]
        for j in range(0, len(idx), 2):          # even rows -= (f/e) * lower odd row
            Vp[idx[j]] = Vp[idx[j]] - fe * _wrapped(Vp, idx, j - 1)
        for j in range(1, len(idx), 2):          # odd rows -= e * modified even row
            Vp[idx[j]] = Vp[idx[j]] - e * Vp[idx[j - 1]]
        if ops is not None:
            ops["reduction_fma"] += len(idx)
            ops["reduction_shuffle"] += 1
    Y = np.zeros_like(V)
    if terminal == "block":                      # eq. cr_terminal_block by block filtering
        h = toeplitz_impulse(eT, fT, L)
        H = np.zeros((L, L))
        for r in range(L):
            H[r, :r + 1] = h[r::-1]
        Y[N - 1] = H @ Vp[N - 1]
    else:                                        # the sequential recurrence (footnote)
        y = np.zeros(L)
        for l in range(L):
            acc = Vp[N - 1][l]
            if l >= 1:
                acc -= eT * y[l - 1]
            if l >= 2:
                acc -= fT * y[l - 2]
            y[l] = acc
        Y[N - 1] = y
    if ops is not None:
        ops["terminal_fma"] += L
    for i in reversed(range(levels)):            # back substitution
        s = 1 << i
        idx = [s * (j + 1) - 1 for j in range(N // s)]
        c, d = rows[i][0], rows[i][1]
        for j in range(0, len(idx), 2):
            Y[idx[j]] = Vp[idx[j]] - c * _wrapped(Y, idx, j - 1) - d * _wrapped(Y, idx, j - 3)
        if ops is not None:
            ops["backsub_fma"] += len(idx)
            ops["backsub_shuffle"] += 1
    if ops is not None:
        ops["backsub_shuffle"] += 1              # the extra R^2 of eq. cr_companion_block
    return Y


# --------------------------------------------------------------------------
# whole signal: cascade on the permuted layout, group after group
# --------------------------------------------------------------------------

def normalise(sos):
    """Rows divided by a0; b0 factored out when every b0 != 0 (eq.
    simple_second_order).  Returns (rows [K][5] = b0 b1 b2 a1 a2, gain)."""
    s = np.asarray(sos, dtype=np.float64)
    rows = []
    for r in s:
        a0 = r[3]
        rows.append([r[0] / a0, r[1] / a0, r[2] / a0, r[4] / a0, r[5] / a0])
    rows = np.array(rows)
    gain = 1.0
    if np.all(rows[:, 0] != 0.0):
        gain = float(np.prod(rows[:, 0]))
        rows[:, 1] /= rows[:, 0]
        rows[:, 2] /= rows[:, 0]
        rows[:, 0] = 1.0
    return rows, gain


def filter_groups(x, sos, N: int, L: int, solver: str = "ph",
                  dtype=np.float64, ops: Counter | None = None):
    """Filter x through the cascade with the multi-block method, one signal
    block group after another, carrying each section's (x[-2], x[-1],
    y[-2], y[-1]) from group to group; zero initial state; the tail is
    zero-padded to a whole group and cut off again."""
    rows, gain = normalise(sos)
    rows = rows.astype(dtype)
    K = rows.shape[0]
    n = len(x)
    G = (n + N * L - 1) // (N * L)
    xp = np.zeros(G * N * L, dtype=dtype)
    xp[:n] = np.asarray(x, dtype=dtype)
    out = np.empty_like(xp)
    xs = np.zeros((K, 2), dtype=dtype)
    ys = np.zeros((K, 2), dtype=dtype)
    for g in range(G):
        X = strided_blocks(xp[g * N * L:(g + 1) * N * L], N, L)   # one permutation
        for k in range(K):
            b0, b1, b2, a1, a2 = rows[k]
            V = nonrecursive_stage(X, b0, b1, b2, a1, a2, xs[k], ys[k], ops)
            xs[k] = (X[N - 2][L - 1], X[N - 1][L - 1])
            Y = (ph_solve if solver == "ph" else cr_solve)(V, a1, a2, ops)
            ys[k] = (Y[N - 2][L - 1], Y[N - 1][L - 1])
            X = Y
        out[g * N * L:(g + 1) * N * L] = unstrided(X) * np.asarray(gain, dtype=dtype)
    return out[:n]


# --------------------------------------------------------------------------
# dense forms (Sections III and V) for brute-force checks on tiny inputs
# --------------------------------------------------------------------------

def dense_banded(c1: float, c2: float, n: int) -> np.ndarray:
    """Unit lower-triangular banded Toeplitz matrix of eq. filtering_AB."""
    M = np.eye(n)
    for i in range(1, n):
        M[i, i - 1] = c1
    for i in range(2, n):
        M[i, i - 2] = c2
    return M


def dense_multiblock(c1: float, c2: float, N: int, L: int):
    """The permuted NL x NL matrix of eq. multi_block_A (blocks are c I on the
    sub-diagonals and c R in the top-right corner) and the NL x 2 terminal
    matrix of eq. multi_block_Am."""
    I = np.eye(L)
    Rm = np.zeros((L, L))
    for i in range(1, L):
        Rm[i, i - 1] = 1.0
    A = np.zeros((N * L, N * L))
    blk = lambda r, c: (slice(r * L, (r + 1) * L), slice(c * L, (c + 1) * L))
    for m in range(N):
        A[blk(m, m)] = I
        for t, cc in ((1, c1), (2, c2)):
            j = m - t
            if j >= 0:
                A[blk(m, j)] = cc * I
            else:
                A[blk(m, j + N)] += cc * Rm
    Am = np.zeros((N * L, 2))
    e0 = np.zeros(L); e0[0] = 1.0
    Am[0:L, 0] = c2 * e0
    Am[0:L, 1] = c1 * e0
    if N > 1:
        Am[L:2 * L, 1] = c2 * e0
    return A, Am
