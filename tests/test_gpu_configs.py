"""GPU parity at the workloads' own sizes and right-hand-side counts.

* Right-hand sides beyond one 16-column tile (17, 32, 33, 64): the tiled
  forward sweep and back substitution of 16 x 16 and 32 x 32 blocks with two
  tiles per workgroup, alone and batched.
* The BABD trapezoid workload (m = 16, N = 262144 steps) at full size, in
  FP64 and with FP32 factors and FP64 refinement.
* A subset of the batched workload drawn with its full law (m in
  {4, 8, 16, 32}, N log-uniform up to 2^16, 1..64 right-hand sides), in FP64
  and FP32 + refinement.
* One request of the serving law at N = 2^20 through the request scheduler,
  and a repeat right-hand side on its kept factor.

Every result meets eta <= 1e-12 and the forward-error bound of tests/_gpu.py
against the oracle."""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle
from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

from . import _gpu as G
from .test_gpu_batch import _alone, _check_against_alone_and_oracle, _device, _systems

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def _say(*a):
    print(*a, flush=True)


# --------------------------------------------------------------------------
# wide right-hand sides: two 16-column tiles per workgroup
@pytest.mark.parametrize("nrhs", [17, 32, 33, 64])
@pytest.mark.parametrize("kind,m,nb,p", [("btri", 32, 300, 0), ("btri", 32, 41, 5),
                                         ("btri", 16, 700, 0), ("btri", 27, 90, 0),
                                         ("babd", 16, 500, 0), ("babd", 32, 120, 0),
                                         ("babd", 12, 77, 3)])
def test_tiled_solves_wide_rhs(kind, m, nb, p, nrhs):
    """pf_solve and pf_factor_solve with more than 16 right-hand sides on
    the matrix-core solve kernels (the 32-column tiles for nrhs > 16)."""
    import torch
    seed = 2100 + nb + 3 * m + nrhs + p
    s = wl.random_btri(nb, m, seed=seed) if kind == "btri" else wl.random_babd(nb, m, seed=seed)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nb * m, nrhs))
    A, keep = G.to_device(s)
    F = pf.pf_factor(A, pf.make_opts(partitions=p))
    try:
        fd = G.rhs_to_device(f)
        x = torch.full_like(fd, np.nan)
        _say(kind, "m", m, "nb", nb, "p", p, "nrhs", nrhs)
        info = pf.pf_solve(F, fd, x)
        assert info.status == 0
        G.check(s, x.cpu().numpy().T, f=f, tag=f"solve {kind} m={m} nb={nb} k={nrhs}")
        x2 = torch.full_like(fd, np.nan)
        assert pf.pf_factor_solve(F, fd, x2).status == 0
        G.check(s, x2.cpu().numpy().T, f=f, tag=f"factor_solve {kind} m={m} nb={nb} k={nrhs}")
    finally:
        pf.pf_destroy(F)
    del keep


def test_batch_tiled_solves_wide_rhs():
    """A batch whose 16 x 16 and 32 x 32 members carry 1..64 right-hand sides
    (one and two tiles per workgroup in the same launches) equals the same
    solves made alone, bit for bit, and the oracle."""
    import torch
    specs = [("btri", 32, 200, 64, 3101), ("btri", 32, 90, 17, 3102), ("btri", 16, 400, 33, 3103),
             ("btri", 16, 150, 16, 3104), ("babd", 16, 300, 40, 3105), ("babd", 32, 60, 21, 3106),
             ("btri", 32, 77, 1, 3107), ("btri", 8, 500, 64, 3108), ("btri", 27, 50, 35, 3109),
             ("babd", 12, 99, 64, 3110)]
    systems = _systems(specs)
    mats, keep, fs, xs = _device(systems)
    _say("batch wide", [(k, m, nb, r) for k, m, nb, r, _ in specs])
    infos, _ = pf.pf_solve_batch(mats, None, [f.shape[0] for _, f in systems], fs, xs)
    torch.cuda.synchronize()
    assert [i.status for i in infos] == [0] * len(systems)
    _check_against_alone_and_oracle(systems, mats, fs, xs, None, "wide")
    del keep


# --------------------------------------------------------------------------
# BABD trapezoid workload at full size
@pytest.fixture(scope="module")
def babd_full():
    s = wl.trapezoid_babd(N=262144, m=16)
    _say("babd full: oracle solve and condition estimate")
    xo = oracle.babd_solve(s.D, s.Lo, s.C, s.f)
    kap = G.kappa(s)
    return s, xo, kap


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
def test_babd_trapezoid_full(babd_full, prec):
    """m = 16, N = 262144 steps (nb = 262145) with the planner's partitions,
    in FP64 and with FP32 factors and FP64 refinement."""
    s, xo, kap = babd_full
    opts = pf.make_opts(prec=pf.PF_FP32_IR if prec == "fp32ir" else pf.PF_FP64)
    _say("babd full", prec)
    x, info, levels = G.gpu_solve(s, opts)
    _say(prec, info.as_dict(), levels)
    assert info.status == 0
    if prec == "fp32ir":
        assert info.eta <= G.ETA_TOL and info.refine_iters >= 1
    _say(G.check(s, x, xref=xo, kap=kap, tag=f"babd full {prec}"))


# --------------------------------------------------------------------------
# the batched workload's law
def _oracle_refs(systems):
    """Per system: kappa and the oracle's solution of right-hand side 0
    (threads: the oracle's C calls release the interpreter lock)."""
    def one(sf):
        s, f = sf
        return G.kappa(s), G.oracle_solve(s, f[0])
    with cf.ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(one, systems))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
def test_batch_workload_law_subset(prec):
    """32 systems drawn with the batched workload's full law (block sizes 4,
    8, 16, 32; N log-uniform on [2^8, 2^16]; 1..64 right-hand sides), solved
    as one batch.  Every right-hand side is held to eta <= 1e-12 (FP64
    residual by the oracle); right-hand side 0 is compared with the oracle's
    solution (kappa from the oracle's estimator)."""
    import torch
    specs = wl.batch_specs(count=32, seed=wl.seed_for(4, 7))
    _say("law subset", prec, [(m, nb, k) for m, nb, k, _ in specs])
    systems = []
    with cf.ThreadPoolExecutor(THREADS) as ex:
        def gen(sp):
            m, nb, k, seed = sp
            s = wl.random_btri(nb, m, seed=seed, manufactured=False)
            f = np.random.default_rng(seed + 1).standard_normal((k, nb * m))
            return s, f
        systems = list(ex.map(gen, specs))
    mats, keep, fs, xs = _device(systems)
    opts = pf.make_opts(prec=pf.PF_FP32_IR if prec == "fp32ir" else pf.PF_FP64)
    infos, _ = pf.pf_solve_batch(mats, opts, [k for _, _, k, _ in specs], fs, xs)
    torch.cuda.synchronize()
    _say("batch done", [i.status for i in infos])
    assert [i.status for i in infos] == [0] * len(systems)
    xh = [x.cpu().numpy() for x in xs]
    del mats, keep, fs, xs
    refs = _oracle_refs(systems)

    def eta_all(i):
        s, f = systems[i]
        r = oracle.btri_residual(s.D, s.Lo, s.Up, f.T, xh[i].T)
        return float(np.max(oracle.eta(oracle.btri_norminf(s.D, s.Lo, s.Up), f.T, xh[i].T, r)))
    with cf.ThreadPoolExecutor(THREADS) as ex:
        etas = list(ex.map(eta_all, range(len(systems))))
    worst = 0.0
    for i, ((s, f), (kap, x0), e) in enumerate(zip(systems, refs, etas)):
        assert e <= G.ETA_TOL, f"sys {i} m={s.m} nb={s.nb}: eta {e:.3e}"
        fe = G.fwd_err(xh[i][0], x0)
        bound = 2e3 * kap * G.EPS
        assert fe <= bound, f"sys {i} m={s.m} nb={s.nb}: forward error {fe:.3e} > {bound:.3e}"
        worst = max(worst, fe / bound)
        if prec == "fp32ir":
            assert infos[i].eta <= G.ETA_TOL and infos[i].refine_iters >= 1
    _say("law subset", prec, "max eta", max(etas), "worst fwd/bound", worst,
         "refine iters", sorted({i.refine_iters for i in infos}))


# --------------------------------------------------------------------------
# one request of the serving law at its largest block count
@pytest.mark.timeout(600)
def test_serving_request_n_2_20():
    """A request with m = 8 and N = 2^20 block rows (the serving law's upper
    clamp) through the request scheduler, then a repeat right-hand side on
    its kept factor; both against the oracle."""
    import torch
    nb, m = 2 ** 20, 8
    s = wl.random_btri(nb, m, seed=wl.seed_for(5, 9), manufactured=True)
    A, keep = G.to_device(s)
    rng = np.random.default_rng(5)
    f2 = rng.standard_normal(s.n)
    S = pf.Server(int(64e9), max_inflight=4, nstreams=2)
    try:
        fd = G.rhs_to_device(s.f)
        x = torch.full_like(fd, np.nan)
        _say("serving nb=2^20 new request")
        t = S.submit(A, fd, x, keep=True)
        info = S.wait(t)
        assert info.status == 0
        f2d = G.rhs_to_device(f2)
        x2 = torch.full_like(f2d, np.nan)
        _say("serving nb=2^20 repeat request")
        t2 = S.submit(A, f2d, x2, factor=t)
        assert S.wait(t2).status == 0
        xa, xb = x.cpu().numpy()[0], x2.cpu().numpy()[0]
    finally:
        S.destroy()
    del keep
    with cf.ThreadPoolExecutor(2) as ex:
        fk = ex.submit(G.kappa, s)
        fo = ex.submit(G.oracle_solve, s, f2)
        kap, xo2 = fk.result(), fo.result()
    _say("new", G.check(s, xa, kap=kap, tag="serving 2^20 new"))
    _say("repeat", G.check(s, xb, f=f2, xref=xo2, kap=kap, tag="serving 2^20 repeat"))
