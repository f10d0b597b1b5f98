"""GPU parity of the scalar tridiagonal kernels (m = 1, FP64) that stage each
workgroup's rows through LDS.

They run the segment mapping's arithmetic in the same order, so every result
must equal the segment kernels' (PF_FLAG_MAP_SEGMENTS) bit for bit: the
solution, the stored factors (a later solve reuses them) and the zero-pivot
report.  Each result is also held to the oracle's acceptance bounds.  Cases
span one partition, ragged partition lengths, several workgroups, levels
whose chains are too long for the LDS arrays (the segment kernels run
those), and the full-size workload law."""
import numpy as np
import pytest

from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

from . import _gpu as G

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def cr_eligible(nb, p):
    """Whether pf_factor_solve with one right-hand side takes the one-launch
    local cyclic reduction (systems that fit one workgroup's LDS)."""
    return 2 <= nb <= 4096 and 1 <= p <= 64 and p <= (nb + 1) // 2


def _run(s, f, opts, split):
    import torch
    A, keep = G.to_device(s)
    F = pf.pf_factor(A, opts)
    try:
        fd = G.rhs_to_device(f)
        x = torch.full_like(fd, np.nan)
        if split:
            pf.pf_refactor(F)
            info = pf.pf_solve(F, fd, x)
        else:
            info = pf.pf_factor_solve(F, fd, x)
        torch.cuda.synchronize()
        levels = pf.pf_factor_levels(F)
    finally:
        pf.pf_destroy(F)
    del keep
    return x.cpu().numpy(), info, levels


# (nb, finest-level p or 0 for the planner, finest-level chain length or 0)
CASES = [(2, 1, 0), (3, 1, 0), (5, 2, 0), (40, 0, 0), (129, 0, 0), (1000, 100, 0),
         (4096, 0, 0), (4099, 1000, 0), (10007, 0, 0), (65537, 0, 0), (70001, 0, 5),
         (70001, 0, 17), (70001, 0, 18), (4096, 16, 0)]


@pytest.mark.parametrize("nb,p,br", CASES)
@pytest.mark.parametrize("split", [False, True])
def test_tridiag_equals_segments(nb, p, br, split):
    s = wl.scalar_tridiagonal(nb, seed=wl.seed_for(1, nb % 97))
    f = s.f.reshape(-1, 1)
    _say("tridiag", nb, p, br, "split" if split else "fused")
    base = dict(partitions=p, block_rows=br)
    x, info, levels = _run(s, f, pf.make_opts(**base), split)
    xs, infos, levs = _run(s, f, pf.make_opts(flags=pf.PF_FLAG_MAP_SEGMENTS, **base), split)
    assert info.status == 0 and infos.status == 0
    assert levels == levs
    if p:
        assert levels[0][2] == p
    if not split and cr_eligible(nb, levels[0][2]):
        # one launch of local cyclic reduction: another elimination order
        assert np.abs(x - xs).max() <= 1e-13 * np.abs(xs).max()
    else:
        assert np.array_equal(x, xs), np.abs(x - xs).max()
    G.check(s, x[0], tag=f"tridiag nb={nb} p={p} br={br}")


@pytest.mark.parametrize("nrhs", [2, 5])
def test_tridiag_multi_rhs(nrhs):
    """Several right-hand sides: the forward and back sweeps of the segment
    mapping read the factors the LDS-staged factor kernel wrote."""
    s = wl.scalar_tridiagonal(30011, seed=wl.seed_for(1, 40 + nrhs))
    rng = np.random.default_rng(nrhs)
    f = rng.standard_normal((s.nb, nrhs))
    x, info, _ = _run(s, f, None, True)
    xs, infos, _ = _run(s, f, pf.make_opts(flags=pf.PF_FLAG_MAP_SEGMENTS), True)
    assert info.status == 0
    assert np.array_equal(x, xs)
    G.check(s, x.T, f=f, tag=f"tridiag nrhs={nrhs}")


def test_tridiag_reuse_factors():
    """pf_factor_solve leaves factors that a later pf_solve reuses."""
    import torch
    s = wl.scalar_tridiagonal(50003, seed=wl.seed_for(1, 60))
    rng = np.random.default_rng(60)
    A, keep = G.to_device(s)
    F = pf.pf_factor(A, None)
    try:
        f1 = G.rhs_to_device(s.f.reshape(-1, 1))
        x1 = torch.empty_like(f1)
        assert pf.pf_factor_solve(F, f1, x1).status == 0
        f2h = rng.standard_normal((s.nb, 1))
        f2 = G.rhs_to_device(f2h)
        x2 = torch.empty_like(f2)
        assert pf.pf_solve(F, f2, x2).status == 0
        torch.cuda.synchronize()
        G.check(s, x1.cpu().numpy()[0], tag="first")
        G.check(s, x2.cpu().numpy().T, f=f2h, tag="reused factors")
    finally:
        pf.pf_destroy(F)
    del keep


@pytest.mark.parametrize("split", [False, True])
def test_tridiag_zero_pivot(split):
    """An exact zero pivot at the first row of partition 7 (its pivot is the
    unmodified diagonal entry) is reported with that block, as the segment
    kernels report it."""
    nb, p = 1000, 100
    s = wl.scalar_tridiagonal(nb, seed=wl.seed_for(1, 70))
    nint = nb - (p - 1)
    q, rem = divmod(nint, p)
    start7 = 7 * (q + 1) + min(7, rem)
    s.D[start7] = 0.0
    f = s.f.reshape(-1, 1)
    _, info, _ = _run(s, f, pf.make_opts(partitions=p), split)
    _, infos, _ = _run(s, f, pf.make_opts(partitions=p, flags=pf.PF_FLAG_MAP_SEGMENTS), split)
    assert info.status == pf.PF_ESINGULAR
    assert info.bad_level == 0 and info.bad_block == start7
    assert (infos.status, infos.bad_level, infos.bad_block) == (info.status, 0, start7)


def test_tridiag_fp32_ir():
    """FP32 factors at the finest level (segment kernel), FP64 reduced
    levels on the LDS-staged kernels, FP64 refinement."""
    s = wl.scalar_tridiagonal(65537, seed=wl.seed_for(1, 80))
    f = s.f.reshape(-1, 1)
    x, info, _ = _run(s, f, pf.make_opts(prec=pf.PF_FP32_IR), True)
    assert info.status == 0 and info.eta <= G.ETA_TOL
    G.check(s, x[0], tag="tridiag fp32-ir")


def test_tridiag_full_size():
    """2^22 unknowns, the planner's levels (every level on the LDS-staged
    kernels)."""
    s = wl.scalar_tridiagonal(1 << 22, seed=wl.seed_for(1, 90))
    f = s.f.reshape(-1, 1)
    x, info, levels = _run(s, f, None, False)
    assert info.status == 0
    _say("levels", levels)
    G.check(s, x[0], tag="tridiag 2^22")
