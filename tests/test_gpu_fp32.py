"""FP32 block eliminations on the matrix cores (v_mfma_f32_16x16x4f32, FP32
accumulation) with the FP64 reduced separator systems, FP64 residual and FP64
iterative refinement (PF_FP32_IR) for 16 x 16 and 32 x 32 blocks (and sizes
padded to them).

Every refined result meets eta <= 1e-12 and the forward-error bound against
the oracle; the FP32-only solution (the first solve, refinement stopped at
once by a loose tolerance) is reported per case and must sit between FP64
and FP32 accuracy, which shows the finest level really ran in FP32."""
import numpy as np
import pytest

from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

from . import _gpu as G
from .test_gpu_batch import _check_against_alone_and_oracle, _device, _systems

pytestmark = pytest.mark.gpu

CASES = [("btri", 16, 3000, 1), ("btri", 16, 700, 20), ("btri", 32, 500, 3),
         ("btri", 32, 300, 33), ("babd", 16, 2000, 1), ("babd", 16, 500, 17),
         ("btri", 27, 200, 2), ("btri", 12, 400, 5), ("babd", 13, 300, 2)]


def _say(*a):
    print(*a, flush=True)


def _solve(s, f, opts, fused):
    import torch
    A, keep = G.to_device(s)
    F = pf.pf_factor(A, opts)
    try:
        fd = G.rhs_to_device(f)
        x = torch.full_like(fd, np.nan)
        info = (pf.pf_factor_solve if fused else pf.pf_solve)(F, fd, x)
        torch.cuda.synchronize()
    finally:
        pf.pf_destroy(F)
    del keep
    xh = x.cpu().numpy().T
    return (xh[:, 0] if np.ndim(f) == 1 else xh), info


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("kind,m,nb,nrhs", CASES)
def test_fp32_matrix_core_refined(kind, m, nb, nrhs, fused):
    seed = 7300 + nb + m + nrhs
    s = wl.random_btri(nb, m, seed=seed) if kind == "btri" else wl.random_babd(nb, m, seed=seed)
    f = np.random.default_rng(seed).standard_normal((nb * m, nrhs))
    x, info = _solve(s, f, pf.make_opts(prec=pf.PF_FP32_IR), fused)
    _say(kind, m, nb, nrhs, "fused" if fused else "split", info.as_dict())
    assert info.status == 0 and info.refine_iters >= 1 and info.eta <= G.ETA_TOL
    G.check(s, x, f=f, tag=f"fp32ir {kind} m={m} nb={nb} k={nrhs}")


@pytest.mark.parametrize("kind,m,nb", [("btri", 16, 3000), ("btri", 32, 500), ("babd", 16, 2000)])
def test_fp32_only_error(kind, m, nb):
    """The first FP32 solve alone (tol = 1 stops refinement at once): its
    error against the oracle is above FP64 rounding and within FP32's
    bound, so the finest level ran in FP32; refinement then brings it to
    FP64 accuracy."""
    seed = 7400 + nb + m
    s = wl.random_btri(nb, m, seed=seed, manufactured=True) if kind == "btri" else \
        wl.random_babd(nb, m, seed=seed)
    kap = G.kappa(s)
    x0, i0 = _solve(s, s.f, pf.make_opts(prec=pf.PF_FP32_IR, tol=1.0), False)
    assert i0.status == 0 and i0.refine_iters == 0
    e32 = G.fwd_err(x0, s.x_true)
    x1, i1 = _solve(s, s.f, pf.make_opts(prec=pf.PF_FP32_IR), False)
    e64 = G.fwd_err(x1, s.x_true)
    eps32 = float(np.finfo(np.float32).eps)
    _say(kind, m, nb, "kappa", kap, "fp32-only error", e32, "eta", i0.eta,
         "refined error", e64, "iters", i1.refine_iters)
    assert 1e3 * kap * G.EPS < e32 <= 1e3 * kap * eps32
    assert e64 <= 1e3 * kap * G.EPS and i1.eta <= G.ETA_TOL


def test_fp32_batch_equals_alone():
    """A PF_FP32_IR batch whose 16 x 16 and 32 x 32 members factor on the FP32
    matrix cores equals the same systems refined alone, bit for bit."""
    import torch
    specs = [("btri", 32, 200, 5, 7501), ("btri", 16, 900, 1, 7502), ("babd", 16, 400, 3, 7503),
             ("btri", 32, 64, 40, 7504), ("btri", 8, 500, 2, 7505), ("btri", 24, 100, 1, 7506)]
    systems = _systems(specs)
    mats, keep, fs, xs = _device(systems)
    opts = pf.make_opts(prec=pf.PF_FP32_IR)
    _say("fp32 batch", [(k, m, nb, r) for k, m, nb, r, _ in specs])
    infos, _ = pf.pf_solve_batch(mats, opts, [f.shape[0] for _, f in systems], fs, xs)
    torch.cuda.synchronize()
    assert [i.status for i in infos] == [0] * len(systems)
    assert all(i.eta <= G.ETA_TOL and i.refine_iters >= 1 for i in infos)
    _check_against_alone_and_oracle(systems, mats, fs, xs, opts, "fp32 batch")
    del keep


@pytest.mark.parametrize("kind", ["btri", "babd"])
def test_fp32_refinement_stops_on_a_zero_pivot(kind):
    """A zero pivot block makes the FP32 solution non-finite: the refinement
    stops at once (no step mends a non-finite residual) and the status is
    the zero pivot's."""
    s = wl.random_btri(300, 16, seed=77) if kind == "btri" else wl.random_babd(300, 16, seed=77)
    s.D[0 if kind == "btri" else 1] = 0.0   # the first pivot block of partition 0
    x, info, _ = G.gpu_solve(s, pf.make_opts(prec=pf.PF_FP32_IR, partitions=4))
    _say(kind, info.as_dict())
    assert info.status == pf.PF_ESINGULAR
    assert info.refine_iters == 0
