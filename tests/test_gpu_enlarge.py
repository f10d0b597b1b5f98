"""The enlarged reduced system (Sec. 2, the modified factorization after
eq. (redmatr)): where a partition's elimination meets a pivot block that is
singular or ill-conditioned, PF_FLAG_ENLARGE stops the elimination before it
and moves that block row into the reduced system.

Systems with exactly singular and with ill-conditioned pivot blocks (the
generators keep the matrix as a whole regular, the oracle's banded /
structured LU with pivoting across blocks solves them): without the flag the
plain factorization reports PF_ESINGULAR (zero pivots); with it every
result meets eta <= 1e-12 and the forward-error bound, the level's partition
count grows by the failing blocks, and on small cases the exported reduced
matrix equals the dense Schur complement on the enlarged separator set."""
import numpy as np
import pytest

import oracle
from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

from . import _gpu as G
from .test_gpu_structure import _separators

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _system(kind, m, nb, rows, how, seed):
    if kind == "btri":
        return wl.btri_failing_pivots(nb, m, seed, rows, how)
    return wl.babd_failing_pivots(nb, m, seed, rows, how)


CASES = [
    # kind, m, nb, p, failing rows, how
    ("btri", 1, 300, 8, [5, 37, 100, 103, 250], "zero"),
    ("btri", 4, 240, 6, [0, 41, 77, 79, 150], "zero"),
    ("btri", 8, 400, 10, [13, 40, 42, 120, 161, 397], "zero"),
    ("btri", 8, 300, 0, [50, 77, 210], "ill"),
    ("btri", 5, 200, 7, [30, 90], "zero"),
    ("btri", 16, 160, 5, [9, 33, 35, 100], "zero"),
    ("btri", 16, 120, 0, [20, 60], "ill"),
    ("btri", 32, 90, 4, [9, 33, 60], "zero"),
    ("btri", 27, 60, 3, [10, 31], "ill"),
]


@pytest.mark.parametrize("kind,m,nb,p,rows,how", CASES)
def test_enlarged_reduced_system_solves(kind, m, nb, p, rows, how):
    seed = 8100 + nb + m + len(rows)
    s = _system(kind, m, nb, rows, how, seed)
    kap = G.kappa(s)
    _say(kind, m, nb, p, rows, how, "kappa", kap)
    if how == "zero":
        # the plain factorization stops at an exactly zero pivot
        _, info, _ = G.gpu_solve(s, pf.make_opts(partitions=p))
        _say("plain:", info.as_dict())
        assert info.status == pf.PF_ESINGULAR
    x, info, levels = G.gpu_solve(s, pf.make_opts(partitions=p, flags=pf.PF_FLAG_ENLARGE))
    _say("enlarged:", info.as_dict(), levels[:3])
    assert info.status == 0
    plain = pf.pf_plan(G.to_device(s)[0], pf.make_opts(partitions=p))
    inside = [r for r in rows if r not in _separators(kind, nb, plain[0][2])]
    if inside:   # failing rows inside partitions: the finest level gains separators
        assert levels[0][2] >= plain[0][2] + 1
    _say(G.check(s, x, kap=kap, tag=f"enlarged {kind} m={m} {how}"))


@pytest.mark.parametrize("m,how", [(8, "zero"), (16, "zero"), (16, "ill")])
def test_enlarge_babd_reports(m, how):
    """Bidiagonal-plus-corner form: a failing diagonal block stays a diagonal
    block of every reduced matrix (eq. (redmatr1)), so the flag detects and
    reports it (ill-conditioned blocks included) instead of moving it."""
    rows = [17, 61]
    s = wl.babd_failing_pivots(120, m, 8150 + m, rows, how)
    _, info, levels = G.gpu_solve(s, pf.make_opts(partitions=5, flags=pf.PF_FLAG_ENLARGE))
    _say("babd", m, how, info.as_dict(), levels[:2])
    assert info.status == pf.PF_ESINGULAR and info.bad_level == 0 and info.bad_block == 17


@pytest.mark.parametrize("kind,m,nb,p,rows", [("btri", 4, 40, 4, [3, 17, 25]),
                                              ("btri", 8, 30, 3, [0, 12, 21]),
                                              ("btri", 1, 60, 5, [6, 30, 44]),
                                              ("btri", 16, 24, 3, [2, 11])])
def test_enlarged_reduced_matrix_is_schur_complement(kind, m, nb, p, rows):
    """The reduced matrix of the enlarged separator set (the balanced
    separators of p and the failing rows) equals A_ss - A_sI A_II^{-1} A_Is."""
    s = _system(kind, m, nb, rows, "zero", 8200 + nb)
    seps = sorted(set(_separators(kind, nb, p)) | set(rows))
    A, keep = G.to_device(s)
    F = pf.pf_factor(A, pf.make_opts(partitions=p, flags=pf.PF_FLAG_ENLARGE))
    try:
        assert pf.pf_sync_status(F).status == 0
        levels = pf.pf_factor_levels(F)
        assert levels[0][2] == p + len(rows)
        Dr, Lor, Upr = pf.pf_factor_export_reduced(F, 0)
    finally:
        pf.pf_destroy(F)
    if kind == "btri":
        Ad = oracle.btri_dense(s.D, s.Lo, s.Up)
        T = oracle.btri_dense(Dr, Lor, Upr) if len(Dr) > 1 else Dr[0]
    else:
        Ad = oracle.babd_dense(s.D, s.Lo, s.C)
        T = oracle.babd_dense(Dr, Lor, Upr)
    S = oracle.schur_complement(Ad, m, seps)
    err = np.abs(T - S).max() / np.abs(S).max()
    _say(kind, m, nb, p, rows, "enlarged reduced vs Schur", err)
    assert T.shape == S.shape and err <= 1e-12
    del keep


def test_enlarged_handle_refactors_and_solves_again():
    """A handle factored with the enlarged separators keeps them: new values
    with the same failing rows refactor and solve (pf_factor_solve) to the
    oracle's tolerance, several right-hand sides included."""
    import torch
    rows = [11, 50, 52, 130]
    s = wl.btri_failing_pivots(200, 8, 8301, rows, "zero")
    A, keep = G.to_device(s)
    F = pf.pf_factor(A, pf.make_opts(partitions=6, flags=pf.PF_FLAG_ENLARGE))
    try:
        s2 = wl.btri_failing_pivots(200, 8, 8302, rows, "zero")
        for dst, src in zip(keep[:3], (s2.D, s2.Lo, s2.Up)):
            dst.copy_(wl.to_device_blocks(src, G.device()))
        f = np.random.default_rng(3).standard_normal((s2.n, 3))
        fd = G.rhs_to_device(f)
        x = torch.full_like(fd, np.nan)
        info = pf.pf_factor_solve(F, fd, x)
        assert info.status == 0
        G.check(s2, x.cpu().numpy().T, f=f, tag="enlarged refactor")
    finally:
        pf.pf_destroy(F)
    del keep
