"""Helpers shared by the GPU tests: move a seeded system to the device, run
the library through its C ABI, and judge the result against the oracle.

Acceptance (for every solution x^ of A x = f):
  * normwise backward error eta = ||f - A x^|| / (||A|| ||x^|| + ||f||)
    (infinity norms, FP64 residual from the oracle) <= 1e-12;
  * forward error ||x^ - x|| / ||x|| <= 1e3 * kappa_inf(A) * eps, with x the
    manufactured solution when there is one; kappa from the oracle's
    estimator.  Where there is none the reference is the oracle's own solution
    x_o, which carries an error of its own: if both x^ and x_o are within
    1e3 kappa eps of the exact x, the triangle inequality puts them within
    2e3 kappa eps of each other, so that comparison uses the doubled bound
    (it asserts no more than the single bound on each).
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

EPS = float(np.finfo(np.float64).eps)
ETA_TOL = 1e-12


def device():
    import torch
    return torch.device("cuda", 0)


def to_device(s: wl.System):
    import torch
    dev = device()
    D = wl.to_device_blocks(s.D, dev)
    Lo = wl.to_device_blocks(s.Lo, dev)
    Up = wl.to_device_blocks(s.Up, dev) if s.kind == "btri" else None
    C = wl.to_device_blocks(s.C[None], dev) if s.kind == "babd" else None
    kind = pf.PF_BTRI if s.kind == "btri" else pf.PF_BABD
    A = pf.make_matrix(kind, s.m, s.nb, D, Lo, Up, C)
    keep = (D, Lo, Up, C)
    return A, keep


def rhs_to_device(f):
    return wl.to_device_rhs(np.asarray(f), device())


def gpu_solve(s: wl.System, opts=None, f=None):
    """Factor + solve on the GPU; returns (x as numpy shaped like f, info,
    levels)."""
    import torch
    f = s.f if f is None else f
    A, keep = to_device(s)
    F = pf.pf_factor(A, opts)
    try:
        fd = rhs_to_device(f)
        xd = torch.empty_like(fd)
        info = pf.pf_solve(F, fd, xd)
        torch.cuda.synchronize()
        levels = pf.pf_factor_levels(F)
    finally:
        pf.pf_destroy(F)
    x = xd.cpu().numpy().T
    if np.ndim(f) == 1:
        x = x[:, 0]
    del keep
    return np.ascontiguousarray(x), info, levels


def oracle_solve(s: wl.System, f=None):
    f = s.f if f is None else f
    if s.kind == "btri":
        return oracle.btri_solve(s.D, s.Lo, s.Up, f)
    return oracle.babd_solve(s.D, s.Lo, s.C, f)


def eta(s: wl.System, x, f=None):
    f = s.f if f is None else f
    if s.kind == "btri":
        r = oracle.btri_residual(s.D, s.Lo, s.Up, f, x)
        na = oracle.btri_norminf(s.D, s.Lo, s.Up)
    else:
        r = oracle.babd_residual(s.D, s.Lo, s.C, f, x)
        na = oracle.babd_norminf(s.D, s.Lo, s.C)
    return float(np.max(oracle.eta(na, f, x, r)))


def kappa(s: wl.System):
    if s.kind == "btri":
        return oracle.btri_condest(s.D, s.Lo, s.Up)
    return oracle.babd_condest(s.D, s.Lo, s.C)


def fwd_err(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def check(s: wl.System, x, f=None, xref=None, kap=None, tag=""):
    """Assert the acceptance bounds; returns a dict of the measured values."""
    f = s.f if f is None else f
    e = eta(s, x, f)
    kap = kappa(s) if kap is None else kap
    if xref is None and s.x_true is not None and f is s.f:
        xref, bound = s.x_true, 1e3 * kap * EPS
    else:
        if xref is None:
            xref = oracle_solve(s, f)
        bound = 2e3 * kap * EPS
    fe = fwd_err(x, xref)
    assert np.all(np.isfinite(x)), f"{tag}: non-finite solution"
    assert e <= ETA_TOL, f"{tag}: eta {e:.3e} > {ETA_TOL}"
    assert fe <= bound, f"{tag}: forward error {fe:.3e} > {bound:.3e} (kappa {kap:.3e})"
    return {"eta": e, "fwd": fe, "bound": bound, "kappa": kap}
