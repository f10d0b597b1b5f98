"""The factor-and-solve entry point that allocates no device memory
(pf_factor_solve_static, its workspace a static device array) against the
allocating path it is a variant of (pf_factor followed by pf_factor_solve):
results equal bit for bit, on two calls in a row, the second smaller, in
both precisions; a system beyond the static workspace is refused before any
device work."""
import ctypes

import numpy as np
import pytest

from paper_0912_3678_amd import pf

from . import _gpu as G
from .test_gpu_batch import _device, _systems

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _allocating(A, fd, opts):
    import torch
    x = torch.full_like(fd, np.nan)
    F = pf.pf_factor(A, opts)
    try:
        info = pf.pf_factor_solve(F, fd, x)
        torch.cuda.synchronize()
    finally:
        pf.pf_destroy(F)
    return x, info


@pytest.mark.parametrize("prec", [pf.PF_FP64, pf.PF_FP32_IR])
def test_static_equals_allocating_two_calls(prec):
    """Two calls in a row (the second with a smaller system, so stale
    contents of the workspace from the first are around) equal the
    allocating factor-and-solve bit for bit and meet the oracle's bounds."""
    import torch
    opts = pf.make_opts(prec=prec)
    specs = [("btri", 8, 20000, 2, 501), ("btri", 8, 3000, 1, 502),
             ("babd", 16, 2500, 1, 503), ("btri", 32, 300, 17, 504), ("btri", 1, 5000, 1, 505),
             ("btri", 5, 700, 3, 506)]
    systems = _systems(specs)
    mats, keep, fs, xs = _device(systems)
    for (s, f), A, fd, xd in zip(systems, mats, fs, xs):
        _say("static", s.kind, s.m, s.nb, f.shape[0], prec)
        info = pf.pf_factor_solve_static(A, fd, xd, opts)
        torch.cuda.synchronize()
        assert info.status == 0, info.as_dict()
        xa, ia = _allocating(A, fd, opts)
        assert ia.status == 0
        assert np.array_equal(xd.cpu().numpy(), xa.cpu().numpy()), f"{s.kind} m={s.m} nb={s.nb}"
        if prec == pf.PF_FP32_IR:
            assert info.refine_iters == ia.refine_iters and info.eta == ia.eta
        G.check(s, xd.cpu().numpy().T, f=f.T, tag=f"static {s.kind} m={s.m} nb={s.nb}")
    del keep


def test_static_asynchronous_in_order_on_one_stream():
    """Without info the FP64 call only queues kernels: two calls queued
    back to back on one stream (the second smaller) give the allocating
    path's results, once the stream is synchronized."""
    import torch
    systems = _systems([("btri", 16, 4000, 1, 511), ("btri", 16, 900, 2, 512)])
    mats, keep, fs, xs = _device(systems)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        assert pf.pf_factor_solve_static(mats[0], fs[0], xs[0], stream=st, want_info=False) is None
        x0 = xs[0].clone()   # ordered on st after the first call, before the second
        assert pf.pf_factor_solve_static(mats[1], fs[1], xs[1], stream=st, want_info=False) is None
    st.synchronize()
    for i, xd in enumerate((x0, xs[1])):
        xa, _ = _allocating(mats[i], fs[i], None)
        assert np.array_equal(xd.cpu().numpy(), xa.cpu().numpy()), f"call {i}"
    del keep


def test_static_refuses_too_big():
    """A plan needing more than the static workspace is PF_ETOOBIG, found on
    the host from the plan alone (the matrix pointers are never read)."""
    lib = pf.load()
    fake = 256
    A = pf.pf_matrix(pf.PF_BTRI, 32, 200000, fake, fake, fake, None)
    rc = lib.pf_factor_solve_static(ctypes.byref(A), None, 1, ctypes.c_void_p(fake), 32 * 200000,
                                    ctypes.c_void_p(fake), 32 * 200000, None, None)
    assert rc == pf.PF_ETOOBIG
    assert lib.pf_factor_solve_static(ctypes.byref(A), None, -1, None, 1, None, 1, None,
                                      None) == -3
