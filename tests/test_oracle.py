"""Pins for the CPU oracle (no GPU).

Each routine of ``oracle/`` is checked against something other than itself:
exact rational arithmetic (brute force), LAPACK through scipy (a library
routine), closed forms (discrete Poisson, scalar trapezoid decay) and plain
step-by-step recurrences (sequential time stepping, a textbook cyclic
reduction step).  The cases are chosen so that a dropped term, a wrong sign
or index, or a transposed operand anywhere in the oracle fails one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import exact
from paper_0912_3678_amd import workloads as wl

EPS = np.finfo(np.float64).eps


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


# --------------------------------------------------------------------------
# exact rational solver: itself pinned by substitution
def test_exact_solver_substitution():
    rng = np.random.default_rng(1)
    A = rng.integers(-5, 6, (6, 6)).tolist()
    A[0][0] = 0  # forces a row interchange
    b = rng.integers(-9, 10, 6).tolist()
    x = exact.solve(A, b)
    for i in range(6):
        assert sum(Fraction(A[i][j]) * x[j] for j in range(6)) == b[i]


# --------------------------------------------------------------------------
# dense LU with partial pivoting
@pytest.mark.parametrize("seed", [2, 3, 4])
def test_dense_vs_exact(oracle, seed):
    rng = np.random.default_rng(seed)
    A = rng.integers(-7, 8, (6, 6))
    A[0, 0] = 0
    A[1, 1] = 0
    b = rng.integers(-9, 10, 6)
    xe = np.array([float(v) for v in exact.solve(A.tolist(), b.tolist())])
    x = oracle.dense_solve(A.astype(float), b.astype(float))
    assert _rel(x, xe) < 1e-12


def test_dense_vs_lapack_and_transpose(oracle):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((60, 60))
    F = rng.standard_normal((60, 3))
    x = oracle.dense_solve(A, F)
    lu = sla.lu_factor(A)
    assert _rel(x, sla.lu_solve(lu, F)) < 1e-11


# --------------------------------------------------------------------------
# banded LU (BTRI as a band) with partial pivoting
def _rand_btri(rng, nb, m, diag=0.0):
    D = rng.standard_normal((nb, m, m)) + diag * np.eye(m)
    Lo = rng.standard_normal((nb - 1, m, m))
    Up = rng.standard_normal((nb - 1, m, m))
    return D, Lo, Up


def test_btri_band_vs_exact(oracle):
    rng = np.random.default_rng(6)
    m, nb = 2, 4
    D = rng.integers(-4, 5, (nb, m, m)).astype(float)
    Lo = rng.integers(-4, 5, (nb - 1, m, m)).astype(float)
    Up = rng.integers(-4, 5, (nb - 1, m, m)).astype(float)
    D[0] = [[0, 1], [2, 0]]  # needs pivoting inside and across blocks
    f = rng.integers(-9, 10, m * nb).astype(float)
    A = oracle.btri_dense(D, Lo, Up)
    xe = np.array([float(v) for v in exact.solve(A.astype(int).tolist(), f.astype(int).tolist())])
    assert _rel(oracle.btri_solve(D, Lo, Up, f), xe) < 1e-12


@pytest.mark.parametrize("m,nb", [(1, 40), (3, 25), (8, 12)])
def test_btri_band_vs_scipy_banded(oracle, m, nb):
    rng = np.random.default_rng(7 + m)
    D, Lo, Up = _rand_btri(rng, nb, m)
    A = oracle.btri_dense(D, Lo, Up)
    F = rng.standard_normal((m * nb, 2))
    kl = ku = 2 * m - 1
    n = m * nb
    ab = np.zeros((kl + ku + 1, n))
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            ab[ku + i - j, j] = A[i, j]
    ref = sla.solve_banded((kl, ku), ab, F)
    x = oracle.btri_solve(D, Lo, Up, F)
    assert _rel(x, ref) < 1e-10
    # transposed solve through the same factors
    xt = oracle.btri_solve_trans(D, Lo, Up, F)
    assert _rel(xt, np.linalg.solve(A.T, F)) < 1e-10


def test_poisson_closed_form(oracle):
    """tridiag(-1,2,-1) x = 1  =>  x_i = i (n+1-i) / 2 (1-based i)."""
    n = 4096
    s = wl.poisson(n)
    i = np.arange(1, n + 1, dtype=np.float64)
    xe = i * (n + 1 - i) / 2.0
    x_th = oracle.thomas(s.Lo.ravel(), s.D.ravel(), s.Up.ravel(), s.f)
    x_bd = oracle.btri_solve(s.D, s.Lo, s.Up, s.f)
    assert _rel(x_th, xe) < 1e-9
    assert _rel(x_bd, xe) < 1e-9


def test_poisson_condition_closed_form(oracle):
    """kappa_inf(tridiag(-1,2,-1)) = n (n+2) / 2 for even n."""
    for n in (16, 256, 4096):
        s = wl.poisson(n)
        k = oracle.btri_condest(s.D, s.Lo, s.Up)
        assert abs(k - n * (n + 2) / 2) <= 1e-8 * n * n


def test_thomas_matches_band_on_workload(oracle):
    s = wl.scalar_tridiagonal(512, seed=11)
    x1 = oracle.thomas(s.Lo.ravel(), s.D.ravel(), s.Up.ravel(), s.f)
    x2 = oracle.btri_solve(s.D, s.Lo, s.Up, s.f)
    assert _rel(x1, s.x_true) < 1e-13
    assert _rel(x2, s.x_true) < 1e-13


def test_condest_vs_dense(oracle):
    rng = np.random.default_rng(12)
    for m, nb in [(2, 6), (4, 5)]:
        D, Lo, Up = _rand_btri(rng, nb, m, diag=1.0)
        A = oracle.btri_dense(D, Lo, Up)
        exact_k = np.linalg.norm(A, np.inf) * np.linalg.norm(np.linalg.inv(A), np.inf)
        est = oracle.btri_condest(D, Lo, Up)
        assert est <= exact_k * (1 + 1e-10)
        assert est >= 0.3 * exact_k


# --------------------------------------------------------------------------
# BABD structured elimination
def test_babd_vs_exact(oracle):
    rng = np.random.default_rng(13)
    m, nb = 2, 4
    D = rng.integers(-4, 5, (nb, m, m)).astype(float)
    Lo = rng.integers(-4, 5, (nb - 1, m, m)).astype(float)
    C = rng.integers(-4, 5, (m, m)).astype(float)
    D[0] = [[0, 0], [0, 1]]  # the first pivot must come from block row 1
    f = rng.integers(-9, 10, m * nb).astype(float)
    A = oracle.babd_dense(D, Lo, C)
    xe = np.array([float(v) for v in exact.solve(A.astype(int).tolist(), f.astype(int).tolist())])
    assert _rel(oracle.babd_solve(D, Lo, C, f), xe) < 1e-12


@pytest.mark.parametrize("m,nb", [(1, 7), (3, 6), (5, 9), (4, 2)])
def test_babd_vs_dense_and_transpose(oracle, m, nb):
    rng = np.random.default_rng(14 + m)
    D = rng.standard_normal((nb, m, m))
    Lo = rng.standard_normal((nb - 1, m, m))
    C = rng.standard_normal((m, m))
    A = oracle.babd_dense(D, Lo, C)
    F = rng.standard_normal((m * nb, 3))
    assert _rel(oracle.babd_solve(D, Lo, C, F), np.linalg.solve(A, F)) < 1e-10
    assert _rel(oracle.babd_solve_trans(D, Lo, C, F), np.linalg.solve(A.T, F)) < 1e-10
    exact_k = np.linalg.norm(A, np.inf) * np.linalg.norm(np.linalg.inv(A), np.inf)
    est = oracle.babd_condest(D, Lo, C)
    assert est <= exact_k * (1 + 1e-10) and est >= 0.3 * exact_k


def test_babd_scalar_trapezoid_closed_form(oracle):
    """y' = lam y, trapezoid: y_n = rho^n y_0 with rho = (1+h lam/2)/(1-h lam/2);
    B0 y_0 + B1 y_N = beta  =>  y_0 = (B0 + rho^N B1)^{-1} beta."""
    m, N, lam = 3, 200, -1.5
    h = 1.0 / N
    rng = np.random.default_rng(15)
    B0 = np.eye(m) + 0.3 * rng.standard_normal((m, m))
    B1 = np.eye(m) + 0.3 * rng.standard_normal((m, m))
    beta = rng.standard_normal(m)
    nb = N + 1
    D = np.empty((nb, m, m))
    D[0] = B0
    D[1:] = (1 - 0.5 * h * lam) * np.eye(m)
    Lo = np.broadcast_to(-(1 + 0.5 * h * lam) * np.eye(m), (N, m, m)).copy()
    f = np.zeros(nb * m)
    f[:m] = beta
    rho = (1 + 0.5 * h * lam) / (1 - 0.5 * h * lam)
    y0 = np.linalg.solve(B0 + rho ** N * B1, beta)
    ye = np.concatenate([rho ** k * y0 for k in range(nb)])
    assert _rel(oracle.babd_solve(D, Lo, B1, f), ye) < 1e-12


def test_babd_ivp_equals_time_stepping(oracle):
    """B0 = I, B1 = 0 (eq. (My)): the solve equals sequential stepping
    y_{n+1} = R_n^{-1} (g_n - S_n y_n)."""
    s = wl.ivp_lower_bidiagonal(N=300, m=4, seed=16)
    x = oracle.babd_solve(s.D, s.Lo, s.C, s.f)
    m, nb = s.m, s.nb
    F = s.f.reshape(nb, m)
    y = [F[0]]
    for k in range(nb - 1):
        y.append(np.linalg.solve(s.D[k + 1], F[k + 1] - s.Lo[k] @ y[-1]))
    assert _rel(x, np.concatenate(y)) < 1e-11


# --------------------------------------------------------------------------
# the sequential IVP routine (Sec. 3) behind the time-parallel driver's parity
def test_ivp_trapezoid_scalar_closed_form(oracle):
    """y' = lam y + c: the trapezoid recursion has the closed form
    y_n = r^n (y0 + c/lam) - c/lam, r = (1 + h lam/2) / (1 - h lam/2)
    (the constant -c/lam is a fixed point of every step)."""
    lam, c, y0, h, steps = -1.7, 0.9, 1.3, 0.01, 400
    y = oracle.ivp_trapezoid(np.array([[lam]]), h, np.full((steps + 1, 1), c), np.array([y0]))
    r = (1 + h * lam / 2) / (1 - h * lam / 2)
    n = np.arange(steps + 1)
    ref = r ** n * (y0 + c / lam) - c / lam
    assert _rel(y[:, 0], ref) < 1e-13


def test_ivp_trapezoid_diagonal_decouples(oracle):
    """A diagonal L decouples into scalar problems, each with its closed
    form; a permutation similarity of L permutes the solution's components."""
    lams = np.array([-0.3, -2.0, 0.4])
    c = np.array([0.5, -1.0, 2.0])
    y0 = np.array([1.0, 0.25, -0.5])
    h, steps = 0.02, 250
    y = oracle.ivp_trapezoid(np.diag(lams), h, np.tile(c, (steps + 1, 1)), y0)
    n = np.arange(steps + 1)[:, None]
    r = (1 + h * lams / 2) / (1 - h * lams / 2)
    assert _rel(y, r ** n * (y0 + c / lams) - c / lams) < 1e-13
    P = np.eye(3)[[2, 0, 1]]
    yp = oracle.ivp_trapezoid(P @ np.diag(lams) @ P.T, h, np.tile(P @ c, (steps + 1, 1)), P @ y0)
    assert _rel(yp, y @ P.T) < 1e-15


def test_ivp_trapezoid_second_order(oracle):
    """Against the exact flow exp(L t) y0 of a damped rotation (g = 0), the
    error at t = 1 falls by about 4 when the step halves (the trapezoid rule
    is of order 2); a dropped h/2 or sign would break the order."""
    L = np.array([[-0.5, 2.0], [-2.0, -0.5]])
    y0 = np.array([1.0, -0.5])
    exact_y = sla.expm(L) @ y0
    errs = []
    for steps in (100, 200, 400):
        y = oracle.ivp_trapezoid(L, 1.0 / steps, np.zeros((steps + 1, 2)), y0)
        errs.append(np.abs(y[-1] - exact_y).max())
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2


def test_ivp_trapezoid_equals_structured_solve(oracle):
    """The sequential routine and the structured BABD elimination of the
    assembled eq. (My) system (B0 = I, B1 = 0) give the same solution."""
    L, g, y0, t0, T = wl.ivp_problem(5, 4, 30, seed=17)
    steps = g.shape[0] - 1
    h = (T - t0) / steps
    y = oracle.ivp_trapezoid(L, h, g, y0)
    eye = np.eye(5)
    D = np.concatenate([eye[None], np.repeat((eye - 0.5 * h * L)[None], steps, 0)])
    Lo = np.repeat((-(eye + 0.5 * h * L))[None], steps, 0)
    f = np.concatenate([y0[None], 0.5 * h * (g[:-1] + g[1:])]).reshape(-1)
    x = oracle.babd_solve(D, Lo, np.zeros((5, 5)), f)
    assert _rel(x, y.reshape(-1)) < 1e-12


# --------------------------------------------------------------------------
# residuals and norms
def test_residual_and_norms_vs_dense(oracle):
    rng = np.random.default_rng(17)
    m, nb = 3, 7
    D, Lo, Up = _rand_btri(rng, nb, m)
    C = rng.standard_normal((m, m))
    x = rng.standard_normal((m * nb, 2))
    f = rng.standard_normal((m * nb, 2))
    A = oracle.btri_dense(D, Lo, Up)
    assert _rel(oracle.btri_residual(D, Lo, Up, f, x), f - A @ x) < 1e-14
    assert abs(oracle.btri_norminf(D, Lo, Up) - np.abs(A).sum(1).max()) < 1e-12
    B = oracle.babd_dense(D, Lo, C)
    assert _rel(oracle.babd_residual(D, Lo, C, f, x), f - B @ x) < 1e-14
    assert abs(oracle.babd_norminf(D, Lo, C) - np.abs(B).sum(1).max()) < 1e-12


# --------------------------------------------------------------------------
# Schur complement onto separators (the reduced matrix, eq. (redmatr))
def test_schur_reduced_system_gives_separator_solution(oracle):
    rng = np.random.default_rng(18)
    m, nb = 2, 11
    D, Lo, Up = _rand_btri(rng, nb, m, diag=3.0)
    A = oracle.btri_dense(D, Lo, Up)
    f = rng.standard_normal(m * nb)
    seps = [3, 7]
    S, g = oracle.schur_complement(A, m, seps, f)
    x = np.linalg.solve(A, f)
    xs = np.concatenate([x[b * m:(b + 1) * m] for b in seps])
    assert _rel(np.linalg.solve(S, g), xs) < 1e-12


def test_schur_one_block_partitions_is_cyclic_reduction_step(oracle):
    """With one-block partitions the reduced matrix is one step of block
    odd-even reduction (textbook formulas, written out here)."""
    rng = np.random.default_rng(19)
    m, nb = 3, 9
    D, Lo, Up = _rand_btri(rng, nb, m, diag=4.0)
    A = oracle.btri_dense(D, Lo, Up)
    seps = [1, 3, 5, 7]                  # eliminate the even blocks 0,2,4,6,8
    S = oracle.schur_complement(A, m, seps)
    inv = np.linalg.inv
    for a, s in enumerate(seps):
        Td = D[s] - Lo[s - 1] @ inv(D[s - 1]) @ Up[s - 1] - Up[s] @ inv(D[s + 1]) @ Lo[s]
        assert _rel(S[a * m:(a + 1) * m, a * m:(a + 1) * m], Td) < 1e-12
        if a > 0:
            Tl = -Lo[s - 1] @ inv(D[s - 1]) @ Lo[s - 2]
            Tu = -Up[s - 2] @ inv(D[s - 1]) @ Up[s - 1]
            assert _rel(S[a * m:(a + 1) * m, (a - 1) * m:a * m], Tl) < 1e-12
            assert _rel(S[(a - 1) * m:a * m, a * m:(a + 1) * m], Tu) < 1e-12


# --------------------------------------------------------------------------
# workload structure (generator, not oracle): the regrouped BVP matrix holds
# exactly the rows of the trapezoid steps and the two boundary conditions
def test_trapezoid_btri_regrouping_is_a_row_permutation(oracle):
    N, m = 12, 8
    s = wl.trapezoid_bvp_btri(N=N, m=m, seed=20)
    A = oracle.btri_dense(s.D, s.Lo, s.Up)
    rng = np.random.default_rng(20)
    M0 = rng.standard_normal((m, m)) / math.sqrt(m) - 2 * np.eye(m)
    M1 = rng.standard_normal((m, m)) / math.sqrt(m)
    h = 1.0 / N
    rows = []
    a = m // 2
    Ba = np.zeros((a, (N + 1) * m)); Ba[:, :a] = np.eye(a)
    rows.append(Ba)
    for k in range(N):
        blk = np.zeros((m, (N + 1) * m))
        blk[:, k * m:(k + 1) * m] = -(np.eye(m) + 0.5 * h * (M0 + k * h * M1))
        blk[:, (k + 1) * m:(k + 2) * m] = np.eye(m) - 0.5 * h * (M0 + (k + 1) * h * M1)
        rows.append(blk)
    Bb = np.zeros((m - a, (N + 1) * m)); Bb[:, N * m + a:] = np.eye(m - a)
    rows.append(Bb)
    full = np.vstack(rows)
    key = lambda r: tuple(np.round(r, 12))
    assert sorted(map(key, A)) == sorted(map(key, full))


def test_eta_hand_computed(oracle):
    """The acceptance quantity eta = ||f - A x|| / (||A|| ||x|| + ||f||)
    (infinity norms, per right-hand side) on a 2 x 2 block tridiagonal system
    with m = 1 whose every value is worked out by hand:
    A = [[2, -1], [1, 3]], ||A||_inf = max(2 + 1, 1 + 3) = 4.
      column 0: x = (1, 2),      f = (1, 7):    A x = (0, 7),         r = (1, 0),
                eta = 1 / (4*2 + 7) = 1/15 (both terms of the denominator count);
      column 1: x = (0.5, -0.25), f = (100, 0): A x = (1.25, -0.25),  r = (98.75, 0.25),
                eta = 98.75 / (4*0.5 + 100) = 98.75/102 (||f|| dominates);
      column 2: x = (1000, 0),   f = (0, 1e-3): A x = (2000, 1000),   r = (-2000, -999.999),
                eta = 2000 / (4*1000 + 1e-3) (||A|| ||x|| dominates).
    A wrong axis, a missing norm or a one-norm in place of the max would
    change at least one of the three."""
    D = np.array([[[2.0]], [[3.0]]])
    Lo = np.array([[[1.0]]])
    Up = np.array([[[-1.0]]])
    x = np.array([[1.0, 0.5, 1000.0], [2.0, -0.25, 0.0]])
    f = np.array([[1.0, 100.0, 0.0], [7.0, 0.0, 1e-3]])
    na = oracle.btri_norminf(D, Lo, Up)
    assert na == 4.0
    r = oracle.btri_residual(D, Lo, Up, f, x)
    np.testing.assert_array_equal(r, np.array([[1.0, 98.75, -2000.0], [0.0, 0.25, 1e-3 - 1000.0]]))
    e = oracle.eta(na, f, x, r)
    expect = np.array([1.0 / 15.0, 98.75 / 102.0, 2000.0 / (4000.0 + 1e-3)])
    np.testing.assert_allclose(e, expect, rtol=1e-15, atol=0)
    # one right-hand side as a 1-D vector gives the same value
    e1 = oracle.eta(na, f[:, 1], x[:, 1], r[:, 1])
    assert np.shape(e1) == (1,)
    assert abs(e1[0] - 98.75 / 102.0) <= 1e-15
    # the bidiagonal-plus-corner form: A = [[2, 5], [1, 3]] (corner 5 in the
    # top right), ||A||_inf = 7; x = (1, 1), f = (7, 5): r = (0, 1),
    # eta = 1 / (7 + 7)
    Db = np.array([[[2.0]], [[3.0]]])
    Lb = np.array([[[1.0]]])
    Cb = np.array([[5.0]])
    nab = oracle.babd_norminf(Db, Lb, Cb)
    assert nab == 7.0
    xb = np.array([1.0, 1.0])
    fb = np.array([7.0, 5.0])
    rb = oracle.babd_residual(Db, Lb, Cb, fb, xb)
    np.testing.assert_array_equal(rb, np.array([0.0, 1.0]))
    assert abs(oracle.eta(nab, fb, xb, rb)[0] - 1.0 / 14.0) <= 1e-16
