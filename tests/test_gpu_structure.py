"""GPU checks of the structure mapping kernels (banded and ABD matrices to the
block tridiagonal form, Sec. 2 and Sec. 3) and of the reduced system the
first level produces (eq. (redmatr), (redmatr1)), against dense constructions
and the oracle's Schur complement."""
import math

import numpy as np
import pytest

import oracle
from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

from . import _gpu as G

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _blocks_from_dense(A, m):
    nb = A.shape[0] // m
    D = np.stack([A[k * m:(k + 1) * m, k * m:(k + 1) * m] for k in range(nb)])
    Lo = np.stack([A[(k + 1) * m:(k + 2) * m, k * m:(k + 1) * m] for k in range(nb - 1)])
    Up = np.stack([A[k * m:(k + 1) * m, (k + 1) * m:(k + 2) * m] for k in range(nb - 1)])
    return D, Lo, Up


def _dev_empty_blocks(count, m):
    import torch
    return torch.full((count, m, m), np.nan, dtype=torch.float64, device=G.device())


def _from_dev_blocks(t):
    # column-major device blocks -> math blocks [k, i, j]
    return np.ascontiguousarray(t.cpu().numpy().transpose(0, 2, 1))


@pytest.mark.parametrize("kl,ku,nb", [(3, 2, 50), (1, 1, 400), (2, 4, 33), (0, 3, 20), (5, 0, 7)])
def test_band_to_btri_exact_and_solve(kl, ku, nb):
    import scipy.linalg
    import torch
    m = max(kl, ku, 1)
    n = m * nb
    rng = np.random.default_rng(1000 + 10 * kl + ku)
    A = np.zeros((n, n))
    for d in range(-kl, ku + 1):
        v = rng.uniform(-1, 1, n - abs(d))
        A += np.diag(v, d)
    A += np.diag(2.0 * (kl + ku) + rng.uniform(0, 1, n))
    ldab = kl + ku + 2                      # one spare row: ldab > kl + ku + 1
    ab = np.full((ldab, n), 7.0)            # junk outside the band must be ignored
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            ab[ku + i - j, j] = A[i, j]
    abd = torch.tensor(ab.T.copy().reshape(-1), dtype=torch.float64, device=G.device())
    D, Lo, Up = _dev_empty_blocks(nb, m), _dev_empty_blocks(nb - 1, m), _dev_empty_blocks(nb - 1, m)
    pf.pf_band_to_btri(n, kl, ku, abd, ldab, D, Lo, Up)
    torch.cuda.synchronize()
    De, Loe, Upe = _blocks_from_dense(A, m)
    assert np.array_equal(_from_dev_blocks(D), De)
    assert np.array_equal(_from_dev_blocks(Lo), Loe)
    assert np.array_equal(_from_dev_blocks(Up), Upe)
    # solve the mapped system on the GPU; pin: LAPACK's banded solver
    x_true = rng.standard_normal(n)
    f = A @ x_true
    s = wl.System("btri", De, Loe, Upe, None, f, x_true, {})
    x, info, _ = G.gpu_solve(s)
    assert info.status == 0
    xs = scipy.linalg.solve_banded((kl, ku), ab[:kl + ku + 1], f)
    G.check(s, x, tag=f"band kl={kl} ku={ku}")
    assert G.fwd_err(x, xs) <= 2e3 * G.kappa(s) * G.EPS


@pytest.mark.parametrize("m,qa,N", [(8, 4, 64), (8, 3, 17), (4, 0, 9), (4, 4, 9), (2, 1, 100)])
def test_abd_to_btri_matches_regrouping(m, qa, N):
    import torch
    rng = np.random.default_rng(2000 + m * 10 + qa)
    M0, M1 = wl._ode_coeffs(rng, m)
    S, R, h = wl._trapezoid_steps(M0, M1, N)
    qb = m - qa
    Ba = rng.standard_normal((qa, m)) + np.eye(m)[:qa]
    Bb = rng.standard_normal((qb, m)) + np.eye(m)[qa:]
    dev = G.device()
    cm = lambda a: torch.tensor(np.ascontiguousarray(a.transpose(0, 2, 1)).reshape(-1),
                                dtype=torch.float64, device=dev)
    colmaj = lambda a: torch.tensor(np.asfortranarray(a).reshape(-1, order="F") if a.size else
                                    np.zeros(1), dtype=torch.float64, device=dev)
    D, Lo, Up = _dev_empty_blocks(N + 1, m), _dev_empty_blocks(N, m), _dev_empty_blocks(N, m)
    Sd, Rd, Bad, Bbd = cm(S), cm(R), colmaj(Ba), colmaj(Bb)
    pf.pf_abd_to_btri(m, N, qa, Bad if qa else None, Sd, Rd, Bbd if qb else None, D, Lo, Up)
    torch.cuda.synchronize()
    # the regrouped rows, written out densely
    n = (N + 1) * m
    A = np.zeros((n, n))
    A[0:qa, 0:m] = Ba
    for k in range(N):
        rows_top = slice(k * m + qa, (k + 1) * m)            # last qb rows of step k
        A[rows_top, k * m:(k + 1) * m] = S[k, qa:]
        A[rows_top, (k + 1) * m:(k + 2) * m] = R[k, qa:]
        rows_bot = slice((k + 1) * m, (k + 1) * m + qa)      # first qa rows of step k
        A[rows_bot, k * m:(k + 1) * m] = S[k, :qa]
        A[rows_bot, (k + 1) * m:(k + 2) * m] = R[k, :qa]
    A[N * m + qa:, N * m:] = Bb
    De, Loe, Upe = _blocks_from_dense(A, m)
    assert np.array_equal(_from_dev_blocks(D), De)
    assert np.array_equal(_from_dev_blocks(Lo), Loe)
    assert np.array_equal(_from_dev_blocks(Up), Upe)
    # the ABD system itself: one BC row block, N step rows, one BC row block
    full = np.vstack([np.hstack([Ba, np.zeros((qa, n - m))])] +
                     [np.hstack([np.zeros((m, k * m)), S[k], R[k], np.zeros((m, n - (k + 2) * m))])
                      for k in range(N)] +
                     [np.hstack([np.zeros((qb, n - m)), Bb])])
    key = lambda r: tuple(np.round(r, 13))
    assert sorted(map(key, A)) == sorted(map(key, full))


def test_abd_to_btri_reproduces_trapezoid_workload():
    import torch
    N, m = 256, 8
    s = wl.trapezoid_bvp_btri(N=N, m=m, seed=77)
    rng = np.random.default_rng(77)
    M0, M1 = wl._ode_coeffs(rng, m)
    S, R, h = wl._trapezoid_steps(M0, M1, N)
    a = m // 2
    Ba = np.eye(m)[:a]
    Bb = np.eye(m)[a:]
    dev = G.device()
    cm = lambda x: torch.tensor(np.ascontiguousarray(x.transpose(0, 2, 1)).reshape(-1),
                                dtype=torch.float64, device=dev)
    fm = lambda x: torch.tensor(np.asfortranarray(x).reshape(-1, order="F"), dtype=torch.float64,
                                device=dev)
    D, Lo, Up = _dev_empty_blocks(N + 1, m), _dev_empty_blocks(N, m), _dev_empty_blocks(N, m)
    pf.pf_abd_to_btri(m, N, a, fm(Ba), cm(S), cm(R), fm(Bb), D, Lo, Up)
    torch.cuda.synchronize()
    assert np.array_equal(_from_dev_blocks(D), s.D)
    assert np.array_equal(_from_dev_blocks(Lo), s.Lo)
    assert np.array_equal(_from_dev_blocks(Up), s.Up)


def _separators(kind, nb, p):
    nint = nb - (p - 1) if kind == "btri" else nb - (p + 1)
    q, rem = divmod(nint, p)
    seps = [] if kind == "btri" else [0]
    for i in range(p):
        start = (0 if kind == "btri" else 1) + i * (q + 1) + min(i, rem)
        ln = q + (1 if i < rem else 0)
        if kind == "babd" or i < p - 1:
            seps.append(start + ln)
    return seps


@pytest.mark.parametrize("kind,m,nb,p", [("btri", 4, 40, 5), ("btri", 8, 23, 4), ("btri", 1, 64, 9),
                                         ("btri", 2, 9, 4), ("babd", 4, 40, 5), ("babd", 8, 30, 3),
                                         ("babd", 2, 11, 5)])
def test_reduced_system_is_schur_complement(kind, m, nb, p):
    seed = 3000 + nb + p
    s = wl.random_btri(nb, m, seed=seed) if kind == "btri" else wl.random_babd(nb, m, seed=seed)
    A, keep = G.to_device(s)
    F = pf.pf_factor(A, pf.make_opts(partitions=p))
    try:
        levels = pf.pf_factor_levels(F)
        assert levels[0][2] == p
        Dr, Lor, Upr = pf.pf_factor_export_reduced(F, 0)
    finally:
        pf.pf_destroy(F)
    if kind == "btri":
        Ad = oracle.btri_dense(s.D, s.Lo, s.Up)
        T = oracle.btri_dense(Dr, Lor, Upr) if len(Dr) > 1 else Dr[0]
    else:
        Ad = oracle.babd_dense(s.D, s.Lo, s.C)
        T = oracle.babd_dense(Dr, Lor, Upr)
    S = oracle.schur_complement(Ad, m, _separators(kind, nb, p))
    err = np.abs(T - S).max() / np.abs(S).max()
    _say(kind, m, nb, p, "reduced vs Schur", err)
    assert T.shape == S.shape
    assert err <= 1e-13
    del keep
