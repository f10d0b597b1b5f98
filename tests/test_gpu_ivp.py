"""GPU tests of the time-parallel IVP driver (Sec. 3): the trapezoid
discretization of y' = L y + g(t) built on the device, and its solution over
a coarse mesh of p sub-intervals (the partitions) against the oracle's
sequential stepping."""
import numpy as np
import pytest

import oracle
from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

from . import _gpu as G

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=G.device())


def _L_dev(L):
    return _dev(np.asarray(L).T.reshape(-1))     # column-major m x m


def _system(L, h, steps):
    """The eq. (My) system of the trapezoid rule as blocks (host): D[0] = I,
    D[n] = I - h/2 L, Lo[n-1] = -(I + h/2 L), C = 0."""
    m = L.shape[0]
    eye = np.eye(m)
    D = np.concatenate([eye[None], np.repeat((eye - 0.5 * h * L)[None], steps, 0)])
    Lo = np.repeat((-(eye + 0.5 * h * L))[None], steps, 0)
    return D, Lo, np.zeros((m, m))


def _check_ivp(L, h, g, y0, got, tag):
    """The device solution against the oracle's sequential stepping of the
    same discretization, both solutions of the eq. (My) system: its backward
    error eta <= 1e-12, and the two within 2e3 kappa eps of each other (each
    within 1e3 kappa eps of the exact discrete solution)."""
    steps = g.shape[0] - 1
    D, Lo, C = _system(L, h, steps)
    f = np.concatenate([y0[None], 0.5 * h * (g[:-1] + g[1:])])
    r = oracle.babd_residual(D, Lo, C, f.reshape(-1), got.reshape(-1))
    eta = float(np.max(oracle.eta(oracle.babd_norminf(D, Lo, C), f.reshape(-1), got.reshape(-1), r)))
    kap = oracle.babd_condest(D, Lo, C)
    ref = oracle.ivp_trapezoid(L, h, g, y0)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    bound = 2e3 * kap * G.EPS
    _say(f"   {tag}: eta {eta:.2e}, rel err vs sequential {err:.2e} (bound {bound:.2e}, kappa {kap:.2e})")
    assert eta <= G.ETA_TOL, tag
    assert err <= bound, tag


def test_trapezoid_system_matches_definition():
    """The device-built eq. (My) system equals its definition entry for entry:
    D[0] = I, D[n] = I - h/2 L, Lo = -(I + h/2 L), C = 0, f[0] = y0,
    f[n] = h/2 (g_{n-1} + g_n)."""
    import torch
    m, steps = 5, 37
    L, g, y0, t0, T = wl.ivp_problem(m, 1, steps, seed=3)
    h = (T - t0) / steps
    D = torch.full(((steps + 1) * m * m,), np.nan, dtype=torch.float64, device=G.device())
    Lo = torch.full((steps * m * m,), np.nan, dtype=torch.float64, device=G.device())
    C = torch.full((m * m,), np.nan, dtype=torch.float64, device=G.device())
    f = torch.full(((steps + 1) * m,), np.nan, dtype=torch.float64, device=G.device())
    pf.pf_ivp_trapezoid_system(m, steps, _L_dev(L), h, _dev(g.reshape(-1)), _dev(y0), D, Lo, C, f)
    torch.cuda.synchronize()
    eye = np.eye(m)
    cm = lambda blocks: np.transpose(blocks, (0, 2, 1)).reshape(-1)   # column-major blocks
    Dref = np.concatenate([eye[None], np.repeat((eye - 0.5 * h * L)[None], steps, 0)])
    Loref = np.repeat((-(eye + 0.5 * h * L))[None], steps, 0)
    fref = np.concatenate([y0[None], 0.5 * h * (g[:-1] + g[1:])]).reshape(-1)
    assert np.array_equal(D.cpu().numpy(), cm(Dref))
    assert np.array_equal(Lo.cpu().numpy(), cm(Loref))
    assert np.array_equal(C.cpu().numpy(), np.zeros(m * m))
    assert np.array_equal(f.cpu().numpy(), fref)


@pytest.mark.parametrize("m,p,N", [(1, 1, 2), (1, 4, 50), (4, 8, 100), (8, 64, 40), (16, 16, 33),
                                   (3, 5, 7), (8, 1, 300), (32, 4, 10), (12, 100, 2), (8, 2048, 8)])
def test_ivp_solve_matches_sequential_stepping(m, p, N):
    """The time-parallel solution over p sub-intervals equals the oracle's
    step-by-step solution of the same discretization (up to rounding):
    single and many sub-intervals, two-step sub-intervals, padded block
    sizes, m = 1 and m = 32."""
    import torch
    L, g, y0, t0, T = wl.ivp_problem(m, p, N, seed=100 + m + p + N)
    steps = p * N
    h = (T - t0) / steps
    y = torch.full(((steps + 1) * m,), np.nan, dtype=torch.float64, device=G.device())
    _say("ivp m", m, "p", p, "N", N)
    info = pf.pf_ivp_solve(m, _L_dev(L), t0, T, p, N, _dev(g.reshape(-1)), _dev(y0), y)
    assert info.status == 0
    _check_ivp(L, h, g, y0, y.cpu().numpy().reshape(steps + 1, m), f"m={m} p={p} N={N}")


def test_ivp_solve_partition_invariance_and_fp32_refinement():
    """One sub-interval or 256, and FP32 factors with FP64 refinement, each
    give the sequential solution to the bounds of _check_ivp."""
    import torch
    m, N0 = 8, 4096
    L, g, y0, t0, T = wl.ivp_problem(m, 1, N0, seed=7)
    gd, yd, Ld = _dev(g.reshape(-1)), _dev(y0), _L_dev(L)
    out = {}
    for name, p, opts in (("p1", 1, None), ("p256", 256, None),
                          ("fp32ir", 256, pf.make_opts(prec=pf.PF_FP32_IR))):
        y = torch.full(((N0 + 1) * m,), np.nan, dtype=torch.float64, device=G.device())
        info = pf.pf_ivp_solve(m, Ld, t0, T, p, N0 // p, gd, yd, y, opts=opts)
        assert info.status == 0, name
        out[name] = y.cpu().numpy()
    h = (T - t0) / N0
    for name, y in out.items():
        _check_ivp(L, h, g, y0, y.reshape(N0 + 1, m), name)


def test_ivp_singular_step_matrix_reported():
    """h/2 L with an eigenvalue 1 makes I - h/2 L singular in every step:
    reported as an exactly singular pivot at level 0, first interior block."""
    import torch
    m, p, N = 2, 4, 8
    h = 1.0 / (p * N)         # a power of two: h/2 * 2/h is exactly 1
    L = np.diag([2.0 / h, -1.0])
    g = np.zeros((p * N + 1, m))
    y = torch.zeros(((p * N + 1) * m,), dtype=torch.float64, device=G.device())
    info = pf.pf_ivp_solve(m, _L_dev(L), 0.0, 1.0, p, N, _dev(g.reshape(-1)), _dev(np.ones(m)), y)
    assert info.status == pf.PF_ESINGULAR
    assert info.bad_level == 0 and info.bad_block == 1


def test_ivp_plan_reused_equals_one_shot():
    """A plan solves several IVPs of its shape (new L, g, y0, interval) with
    no allocation, each equal bit for bit to the one-shot pf_ivp_solve and to
    sequential stepping up to rounding."""
    import torch
    m, p, N = 8, 32, 16
    plan = pf.pf_ivp_create(m, p, N)
    try:
        for seed, (t0, T) in ((21, (0.0, 1.0)), (22, (0.5, 2.0)), (23, (-1.0, 0.0))):
            L, g, y0, _, _ = wl.ivp_problem(m, p, N, seed=seed, t0=t0, T=T)
            Ld, gd, y0d = _L_dev(L), _dev(g.reshape(-1)), _dev(y0)
            y1 = torch.full(((p * N + 1) * m,), np.nan, dtype=torch.float64, device=G.device())
            y2 = torch.full_like(y1, np.nan)
            _say("plan run seed", seed)
            assert pf.pf_ivp_run(plan, Ld, t0, T, gd, y0d, y1).status == 0
            assert pf.pf_ivp_solve(m, Ld, t0, T, p, N, gd, y0d, y2).status == 0
            assert torch.equal(y1, y2)
            _check_ivp(L, (T - t0) / (p * N), g, y0, y1.cpu().numpy().reshape(p * N + 1, m),
                       f"plan seed {seed}")
    finally:
        pf.pf_ivp_destroy(plan)


def test_ivp_system_through_pf_factor_equals_driver():
    """The system from pf_ivp_trapezoid_system, factored by pf_factor with the
    sub-intervals as partitions and solved with pf_factor_solve, is the
    driver's computation: the same solution bit for bit."""
    import torch
    m, p, N = 6, 16, 25
    L, g, y0, t0, T = wl.ivp_problem(m, p, N, seed=41)
    steps, nb = p * N, p * N + 1
    h = (T - t0) / steps
    Ld, gd, y0d = _L_dev(L), _dev(g.reshape(-1)), _dev(y0)
    f64 = dict(dtype=torch.float64, device=G.device())
    D, Lo = torch.empty((nb * m * m,), **f64), torch.empty((steps * m * m,), **f64)
    C, f = torch.empty((m * m,), **f64), torch.empty((nb * m,), **f64)
    pf.pf_ivp_trapezoid_system(m, steps, Ld, h, gd, y0d, D, Lo, C, f)
    F = pf.pf_factor(pf.make_matrix(pf.PF_BABD, m, nb, D, Lo, None, C), pf.make_opts(partitions=p))
    try:
        x1 = torch.full((nb * m,), np.nan, **f64)
        assert pf.pf_factor_solve(F, f.view(1, -1), x1.view(1, -1)).status == 0
    finally:
        pf.pf_destroy(F)
    x2 = torch.full((nb * m,), np.nan, **f64)
    assert pf.pf_ivp_solve(m, Ld, t0, T, p, N, gd, y0d, x2).status == 0
    assert torch.equal(x1, x2)
