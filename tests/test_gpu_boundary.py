"""GPU checks of the boundary's ownership and reuse rules: factor memory
from the caller's allocator (PyTorch's caching allocator), and batches
that solve with factors the caller already holds.  Results must equal the
default paths bit for bit and meet the oracle's acceptance bounds."""
import numpy as np
import pytest

from paper_0912_3678_amd import pf

from . import _gpu as G
from .test_gpu_batch import _alone, _check_against_alone_and_oracle, _device, _systems

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("prec", [pf.PF_FP64, pf.PF_FP32_IR])
def test_torch_allocator_backs_factor_memory(prec):
    """With PyTorch's caching allocator set, a handle's memory comes from it
    (torch counts it while the handle lives and gets it back at pf_destroy),
    and the solutions equal those of the default allocator bit for bit."""
    import torch
    specs = [("btri", 8, 900, 2, 401), ("babd", 16, 300, 1, 402), ("btri", 5, 120, 3, 403)]
    systems = _systems(specs)
    mats, keep, fs, xs = _device(systems)
    opts = pf.make_opts(prec=prec)
    ref = [_alone(A, fd, opts) for A, fd in zip(mats, fs)]
    torch.cuda.synchronize()
    live = pf.use_torch_allocator()
    try:
        before = torch.cuda.memory_allocated()
        hs = [pf.pf_factor(A, opts) for A in mats]
        assert len(live) == len(hs)
        held = torch.cuda.memory_allocated() - before
        assert held >= sum(pf.pf_factor_bytes(A, opts) for A in mats)
        for (s, f), F, fd, xd, xr in zip(systems, hs, fs, xs, ref):
            _say("torch allocator", s.kind, s.m, s.nb, f.shape[0], prec)
            info = pf.pf_solve(F, fd, xd)
            assert info.status == 0
            assert np.array_equal(xd.cpu().numpy(), xr.cpu().numpy())
            G.check(s, xd.cpu().numpy().T, f=f.T, tag=f"torch alloc {s.kind} m={s.m}")
        for F in hs:
            pf.pf_destroy(F)
        torch.cuda.synchronize()
        assert not live
        assert torch.cuda.memory_allocated() == before
    finally:
        pf.pf_set_allocator()
    del keep


@pytest.mark.parametrize("prec", [pf.PF_FP64, pf.PF_FP32_IR])
def test_solve_batch_with_existing_factors(prec):
    """pf_solve_batch with some systems' factors passed in (from pf_factor):
    those are solved without refactoring -- one with more right-hand sides
    than its handle's workspace holds -- next to systems the batch factors;
    every result equals the system solved alone, bit for bit, and the
    oracle; the new factors come back and solve again to the same result."""
    import torch
    specs = [("btri", 8, 1000, 1, 411), ("btri", 16, 300, 5, 412), ("babd", 8, 300, 2, 413),
             ("btri", 4, 77, 3, 414), ("babd", 16, 200, 1, 415), ("btri", 32, 60, 20, 416),
             ("btri", 1, 4099, 1, 417), ("btri", 13, 90, 2, 418)]
    systems = _systems(specs)
    mats, keep, fs, xs = _device(systems)
    opts = pf.make_opts(prec=prec)
    # handles from pf_factor hold the workspace of one right-hand side:
    # system 2's two right-hand sides make it grow
    given = [pf.pf_factor(A, opts) if i % 2 == 0 else None for i, A in enumerate(mats)]
    _say("existing factors", prec)
    infos, out = pf.pf_solve_batch(mats, opts, [f.shape[0] for _, f in systems], fs, xs,
                                   factors=given)
    torch.cuda.synchronize()
    try:
        assert [i.status for i in infos] == [0] * len(systems)
        for i, h in enumerate(out):
            assert h is not None and h.value
            if given[i] is not None:
                assert h.value == given[i].value
        _check_against_alone_and_oracle(systems, mats, fs, xs, opts, "existing")
        # the new factors solve again to the same result
        for i, ((s, f), h, fd, xd) in enumerate(zip(systems, out, fs, xs)):
            x2 = torch.full_like(fd, np.nan)
            assert pf.pf_solve(h, fd, x2).status == 0
            assert np.array_equal(x2.cpu().numpy(), xd.cpu().numpy()), f"sys {i}"
    finally:
        for h in out:
            pf.pf_destroy(h)
    del keep


def test_solve_batch_rejects_mismatched_factor():
    """An existing factor of another shape or precision is argument -10."""
    import torch
    systems = _systems([("btri", 8, 100, 1, 421), ("btri", 8, 120, 1, 422)])
    mats, keep, fs, xs = _device(systems)
    F = pf.pf_factor(mats[0])
    try:
        with pytest.raises(pf.PFError) as e:
            pf.pf_solve_batch(mats, None, [1, 1], fs, xs, factors=[None, F])
        assert e.value.code == -10
        with pytest.raises(pf.PFError) as e:
            pf.pf_solve_batch(mats[:1], pf.make_opts(prec=pf.PF_FP32_IR), [1], fs[:1], xs[:1],
                              factors=[F])
        assert e.value.code == -10
        torch.cuda.synchronize()
    finally:
        pf.pf_destroy(F)
    del keep
