"""Small scalar tridiagonal systems in one launch: the finest level's
partitions eliminated by local cyclic reduction (Sec. 2, the cyclic
reduction variant of the local factorization), the reduced system on the
separators by parallel cyclic reduction across one wave's lanes, then the
back substitution (kernels_tri_cr.hip).

Checked against the oracle (Thomas elimination, and the exact solution of
manufactured systems) at the acceptance bounds, against the multi-launch
path of the same partitions, over partition counts 1..64 and ragged
lengths; the stored factors a later pf_solve needs are rebuilt; a zero
pivot is reported with its block."""
import numpy as np
import pytest

import oracle
from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

from . import _gpu as G
from .test_gpu_tridiag import _run, cr_eligible

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("nb,p", [(2, 1), (3, 1), (3, 2), (5, 2), (17, 3), (64, 16), (100, 7),
                                  (255, 4), (1000, 1), (1000, 33), (4095, 64), (4096, 16),
                                  (4096, 0), (4096, 1), (2049, 5)])
def test_tri_cr_one_launch(nb, p):
    s = wl.scalar_tridiagonal(nb, seed=wl.seed_for(1, 200 + nb % 89 + p))
    f = s.f.reshape(-1, 1)
    x, info, levels = _run(s, f, pf.make_opts(partitions=p), False)
    assert cr_eligible(nb, levels[0][2])
    xm, infom, _ = _run(s, f, pf.make_opts(partitions=p, flags=pf.PF_FLAG_MAP_SEGMENTS), False)
    assert info.status == 0 and infom.status == 0
    xo = oracle.thomas(s.Lo.ravel(), s.D.ravel(), s.Up.ravel(), s.f)
    rel = np.abs(x[0] - xo).max() / np.abs(xo).max()
    _say(nb, levels[0][2], "vs Thomas", rel, "vs multi-launch",
         np.abs(x - xm).max() / np.abs(xm).max())
    assert np.abs(x - xm).max() <= 1e-13 * np.abs(xm).max()
    G.check(s, x[0], tag=f"cr nb={nb} p={p}")


@pytest.mark.parametrize("p", [16, 64])
def test_tri_cr_poisson_closed_form(p):
    """The discrete Poisson matrix (tridiag(-1, 2, -1), f = 1) at n = 4096
    with 16 and 64 partitions: x_i = i (n + 1 - i) / 2."""
    s = wl.poisson(4096)
    x, info, levels = _run(s, s.f.reshape(-1, 1), pf.make_opts(partitions=p), False)
    assert info.status == 0 and levels[0][2] == p
    i = np.arange(1, 4097)
    exact = i * (4097 - i) / 2.0
    rel = np.abs(x[0] - exact).max() / exact.max()
    kap = 4096 * 4098 / 2
    _say("poisson", rel, "bound", 1e3 * kap * G.EPS)
    assert rel <= 1e3 * kap * G.EPS


def test_tri_cr_then_solve_refactors():
    """After the one-launch factor-and-solve (which stores no factors), a
    pf_solve with stored factors refactors first; both solutions meet the
    bounds."""
    import torch
    s = wl.scalar_tridiagonal(4096, seed=wl.seed_for(1, 310))
    rng = np.random.default_rng(310)
    A, keep = G.to_device(s)
    F = pf.pf_factor(A, pf.make_opts(partitions=16))
    try:
        # new values behind the handle's pointers, then factor-and-solve
        D2 = s.D * 1.5
        keep[0].copy_(wl.to_device_blocks(D2, G.device()))
        s2 = wl.System("btri", D2, s.Lo, s.Up, None, None)
        f1h = rng.standard_normal(4096)
        f1 = G.rhs_to_device(f1h)
        x1 = torch.empty_like(f1)
        assert pf.pf_factor_solve(F, f1, x1).status == 0
        f2h = rng.standard_normal((4096, 2))
        f2 = G.rhs_to_device(f2h)
        x2 = torch.empty_like(f2)
        assert pf.pf_solve(F, f2, x2).status == 0
        torch.cuda.synchronize()
        G.check(s2, x1.cpu().numpy()[0], f=f1h, tag="cr fused")
        G.check(s2, x2.cpu().numpy().T, f=f2h, tag="solve after cr")
    finally:
        pf.pf_destroy(F)
    del keep


@pytest.mark.parametrize("p", [16, 64])
def test_tri_cr_zero_pivot(p):
    """A zero diagonal entry at the first row of partition 7 (eliminated in
    the first round as it stands) is reported with that block."""
    nb = 4096
    s = wl.scalar_tridiagonal(nb, seed=wl.seed_for(1, 320))
    nint = nb - (p - 1)
    q, rem = divmod(nint, p)
    start7 = 7 * (q + 1) + min(7, rem)
    s.D[start7] = 0.0
    _, info, _ = _run(s, s.f.reshape(-1, 1), pf.make_opts(partitions=p), False)
    assert info.status == pf.PF_ESINGULAR
    assert info.bad_level == 0 and info.bad_block == start7
