"""GPU tests of the request scheduler (continuous batching under a memory
budget, resident factors for repeat right-hand sides) and of the autotuner.

Every request runs the same plan and kernels as the same solve made alone,
so its solution must equal the solo result bit for bit, whatever else was
admitted, queued or evicted around it; each is also held to the oracle's
acceptance bounds."""
import numpy as np
import pytest

from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

from . import _gpu as G

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _rhs(n, k, seed):
    import torch
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, k))
    return f, torch.tensor(np.ascontiguousarray(f.T), dtype=torch.float64, device=G.device())


def _alone_new(A, fd):
    import torch
    x = torch.full_like(fd, np.nan)
    F = pf.pf_factor(A)
    try:
        pf.pf_factor_solve(F, fd, x)
        torch.cuda.synchronize()
    finally:
        pf.pf_destroy(F)
    return x.cpu().numpy()


def _alone_repeat(A, fd):
    import torch
    x = torch.full_like(fd, np.nan)
    F = pf.pf_factor(A)
    try:
        pf.pf_solve(F, fd, x)
        torch.cuda.synchronize()
    finally:
        pf.pf_destroy(F)
    return x.cpu().numpy()


@pytest.mark.parametrize("reserve", [False, True])
def test_serving_mix_equals_alone_with_queueing_and_eviction(reserve):
    """reserve: the request memory is carved from one allocation made up
    front (pf_server_reserve), ranges freed by one request going to the
    next; any overlap between live ranges would corrupt a solution."""
    import torch
    specs = [(8, 3000, 1), (16, 500, 1), (4, 2000, 2), (3, 900, 1), (8, 5000, 1), (32, 40, 1),
             (8, 700, 3), (16, 1200, 1), (2, 4000, 1), (8, 2500, 1)]
    systems = []
    for i, (m, nb, k) in enumerate(specs):
        s = wl.random_btri(nb, m, seed=8000 + i)
        A, keep = G.to_device(s)
        systems.append((s, A, keep, k))
    # a budget that holds only a few systems at once: requests queue, kept
    # factors get evicted
    sizes = [pf.pf_factor_bytes(A) + pf.pf_solve_bytes_per_rhs(A) * k for _, A, _, k in systems]
    budget = int(max(sizes) * 2.5)
    S = pf.Server(budget, max_inflight=4, nstreams=3)
    if reserve:
        S.reserve(budget)
        with pytest.raises(pf.PFError):   # once per server
            S.reserve(1 << 20)
    try:
        reqs = []    # (ticket, system index, f numpy, f device, x device, kind)
        for i, (s, A, keep, k) in enumerate(systems):
            f, fd = _rhs(s.n, k, 100 + i)
            x = torch.full_like(fd, np.nan)
            t = S.submit(A, fd, x, keep=(i % 3 == 0))
            reqs.append((t, i, f, fd, x, "new"))
        # repeats on kept factors (tickets of requests 0, 3, 6, 9), some
        # submitted before their factor's request has finished
        for j, i in enumerate([0, 3, 6, 9, 0]):
            s, A, keep, k = systems[i]
            f, fd = _rhs(s.n, k, 500 + j)
            x = torch.full_like(fd, np.nan)
            t = S.submit(A, fd, x, factor=reqs[i][0])
            reqs.append((t, i, f, fd, x, "repeat"))
        _say("stats after submit", S.stats())
        for t, i, f, fd, x, kind in reqs:
            info = S.wait(t)
            assert info.status == 0, (t, i, info.as_dict())
        st = S.stats()
        _say("stats at end", st)
        assert st["completed"] == len(reqs) and st["queued"] == 0 and st["inflight"] == 0
        for t, i, f, fd, x, kind in reqs:
            s, A, keep, k = systems[i]
            xs = x.cpu().numpy()
            xa = _alone_new(A, fd) if kind == "new" else _alone_repeat(A, fd)
            assert np.array_equal(xs, xa), f"ticket {t} ({kind}, system {i}): mix != alone"
            G.check(s, xs.T, f=f, tag=f"serving ticket {t} {kind} m={s.m} nb={s.nb}")
            sub, start, done = S.times(t)
            assert 0 <= sub and start >= 0 and done >= start, (sub, start, done)
    finally:
        S.destroy()
    torch.cuda.synchronize()


def test_serving_rejects_request_beyond_budget():
    import torch
    s = wl.random_btri(2000, 8, seed=9)
    A, keep = G.to_device(s)
    S = pf.Server(pf.pf_factor_bytes(A) // 2)
    try:
        f, fd = _rhs(s.n, 1, 1)
        x = torch.empty_like(fd)
        with pytest.raises(pf.PFError) as e:
            S.submit(A, fd, x)
        assert e.value.code == pf.PF_ENOMEM
    finally:
        S.destroy()


def test_serving_evicts_idle_factors():
    import torch
    sys3 = [wl.random_btri(3000, 8, seed=20 + i) for i in range(3)]
    devs = [G.to_device(s) for s in sys3]
    one = pf.pf_factor_bytes(devs[0][0]) + pf.pf_solve_bytes_per_rhs(devs[0][0])
    S = pf.Server(int(one * 2.2), max_inflight=1, nstreams=1)
    try:
        tickets = []
        for i, (s, (A, keep)) in enumerate(zip(sys3, devs)):
            f, fd = _rhs(s.n, 1, i)
            x = torch.empty_like(fd)
            t = S.submit(A, fd, x, keep=True)
            S.wait(t)
            tickets.append((t, s, f, x))
        st = S.stats()
        _say(st)
        assert st["evictions"] >= 1 and st["resident"] <= 2
        for t, s, f, x in tickets:
            G.check(s, x.cpu().numpy().T, f=f, tag=f"kept {t}")
        with pytest.raises(pf.PFError):      # the evicted factor is gone
            f, fd = _rhs(sys3[0].n, 1, 9)
            S.submit(devs[0][0], fd, torch.empty_like(fd), factor=tickets[0][0])
    finally:
        S.destroy()


@pytest.mark.parametrize("kind,m,nb", [("btri", 8, 20000), ("babd", 4, 3000)])
def test_autotune_choice_solves(kind, m, nb):
    import torch
    pf.pf_autotune_clear()
    s = wl.random_btri(nb, m, seed=31) if kind == "btri" else wl.random_babd(nb, m, seed=31)
    A, keep = G.to_device(s)
    best, ms = pf.pf_autotune(A)
    _say(kind, m, nb, "tuned", {k: getattr(best, k) for k, _ in best._fields_}, ms)
    assert ms > 0
    x, info, levels = G.gpu_solve(s, best)
    assert info.status == 0
    G.check(s, x, tag="tuned")
    # the cached choice is what PF_FLAG_AUTOTUNE uses
    x2, info2, levels2 = G.gpu_solve(s, pf.make_opts(flags=pf.PF_FLAG_AUTOTUNE))
    assert levels2 == levels
    assert np.array_equal(x, x2)
    del keep


@pytest.mark.parametrize("reserve", [False, True])
def test_serving_fp32_refined_mix_equals_alone(reserve):
    """PF_FP32_IR requests: the refinement runs from the scheduler's polling,
    step for step what pf_solve's loop does, so each solution equals the
    same refined solve made alone bit for bit, with its iteration count and
    eta; repeats on one kept factor take turns on its residual workspace."""
    import torch
    opts = pf.make_opts(prec=pf.PF_FP32_IR)
    specs = [(8, 3000, 1), (16, 500, 2), (4, 2000, 1), (3, 900, 1), (32, 60, 1), (8, 1500, 3)]
    systems = []
    for i, (m, nb, k) in enumerate(specs):
        s = wl.random_btri(nb, m, seed=8100 + i)
        A, keep = G.to_device(s)
        systems.append((s, A, keep, k))
    sizes = [pf.pf_factor_bytes(A, opts) + pf.pf_solve_bytes_per_rhs(A, opts) * k
             for _, A, _, k in systems]
    S = pf.Server(int(max(sizes) * 3), opts, max_inflight=4, nstreams=3)
    if reserve:
        S.reserve(int(max(sizes) * 3))

    def alone(A, fd, repeat):
        x = torch.full_like(fd, np.nan)
        F = pf.pf_factor(A, opts)
        try:
            info = (pf.pf_solve if repeat else pf.pf_factor_solve)(F, fd, x)
        finally:
            pf.pf_destroy(F)
        return x.cpu().numpy(), info

    try:
        reqs = []
        for i, (s, A, keep, k) in enumerate(systems):
            f, fd = _rhs(s.n, k, 300 + i)
            x = torch.full_like(fd, np.nan)
            t = S.submit(A, fd, x, keep=(i % 2 == 0))
            reqs.append((t, i, f, fd, x, False))
        # three repeats on one kept factor, queued behind each other's
        # refinement, and one on another
        for j, i in enumerate([0, 0, 2, 0]):
            s, A, keep, k = systems[i]
            f, fd = _rhs(s.n, k, 700 + j)
            x = torch.full_like(fd, np.nan)
            t = S.submit(A, fd, x, factor=reqs[i][0])
            reqs.append((t, i, f, fd, x, True))
        infos = {}
        for t, *_ in reqs:
            info = S.wait(t)
            assert info.status == 0, (t, info.as_dict())
            infos[t] = info
        st = S.stats()
        _say("stats at end", st)
        assert st["completed"] == len(reqs) and st["inflight"] == 0
        for t, i, f, fd, x, repeat in reqs:
            s, A, keep, k = systems[i]
            xs = x.cpu().numpy()
            xa, ia = alone(A, fd, repeat)
            got = infos[t]
            _say(f"ticket {t} m={s.m} nb={s.nb} repeat={repeat}: iters {got.refine_iters} "
                 f"eta {got.eta:.3e} (alone {ia.refine_iters}, {ia.eta:.3e})")
            assert got.refine_iters == ia.refine_iters and got.eta == ia.eta, t
            assert got.refine_iters >= 1 and got.eta <= 1e-12
            assert np.array_equal(xs, xa), f"ticket {t} (system {i}): mix != alone"
            G.check(s, xs.T, f=f, tag=f"fp32 refined ticket {t} m={s.m} nb={s.nb}")
    finally:
        S.destroy()
    torch.cuda.synchronize()
