"""CPU checks of the C ABI: the library loads, exports every function that
include/pf.h declares, validates arguments on the host, and plans the
recursion as documented (no GPU work is issued)."""
import ctypes
import os
import re

import pytest

from paper_0912_3678_amd import pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    lib = pf.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pf.EXPORTED)


def _mat(kind=pf.PF_BTRI, m=8, nb=65537):
    fake = 256  # never dereferenced by the host-side calls below
    return pf.pf_matrix(kind, m, nb, fake, fake, fake if kind == pf.PF_BTRI else None,
                        fake if kind == pf.PF_BABD else None)


def test_argument_validation():
    lib = pf.load()
    h = ctypes.c_void_p()
    assert lib.pf_factor(None, None, None, ctypes.byref(h)) == -1
    bad = _mat(nb=1)
    assert lib.pf_factor(ctypes.byref(bad), None, None, ctypes.byref(h)) == -1
    mixed = pf.pf_matrix(pf.PF_BTRI, 4, 10, 256, 256, 256, 256)   # BTRI with a corner
    assert lib.pf_factor(ctypes.byref(mixed), None, None, ctypes.byref(h)) == -1
    big = _mat(m=33)
    assert lib.pf_factor(ctypes.byref(big), None, None, ctypes.byref(h)) == pf.PF_EUNSUPPORTED
    A = _mat(nb=11)
    o = pf.make_opts(partitions=7)     # > (nb+1)/2
    assert lib.pf_factor(ctypes.byref(A), ctypes.byref(o), None, ctypes.byref(h)) == -2
    assert lib.pf_factor(ctypes.byref(A), None, None, None) == -4
    assert lib.pf_solve(None, 1, None, 1, None, 1, None, None) == -1
    assert lib.pf_strerror(pf.PF_ESINGULAR).decode().startswith("exactly zero")


def test_ivp_argument_validation():
    """The IVP entry points reject bad arguments on the host, before any
    device allocation or launch."""
    lib = pf.load()
    fake = ctypes.c_void_p(256)   # never dereferenced: every call below fails validation
    ok = dict(m=4, L=fake, t0=0.0, T=1.0, p=8, N=16, g=fake, y0=fake, y=fake)

    def call(**kw):
        a = dict(ok, **kw)
        return lib.pf_ivp_solve(a["m"], a["L"], a["t0"], a["T"], a["p"], a["N"], a["g"],
                                a["y0"], a["y"], None, None, None)
    assert call(m=0) == -1 and call(m=33) == -1
    assert call(L=None) == -2
    assert call(T=0.0) == -4 and call(T=float("nan")) == -4
    assert call(p=0) == -5 and call(p=2 ** 40) == -5
    assert call(N=1) == -6                  # a sub-interval needs two steps (p <= (nb-1)/2)
    assert call(N=2 ** 61) == -6            # p * N would overflow
    assert call(g=None) == -7 and call(y0=None) == -8 and call(y=None) == -9
    h = ctypes.c_void_p()
    assert lib.pf_ivp_create(0, 8, 16, None, None, ctypes.byref(h)) == -1
    assert lib.pf_ivp_create(4, 0, 16, None, None, ctypes.byref(h)) == -2
    assert lib.pf_ivp_create(4, 8, 1, None, None, ctypes.byref(h)) == -3
    assert lib.pf_ivp_create(4, 8, 16, None, None, None) == -6
    assert lib.pf_ivp_run(None, fake, 0.0, 1.0, fake, fake, fake, None, None) == -1
    sysargs = [4, 10, fake, 0.1, fake, fake, fake, fake, fake, fake, None]
    assert lib.pf_ivp_trapezoid_system(0, *sysargs[1:]) == -1
    assert lib.pf_ivp_trapezoid_system(4, 0, *sysargs[2:]) == -2
    assert lib.pf_ivp_trapezoid_system(4, 10, fake, -0.1, *sysargs[4:]) == -4
    assert lib.pf_ivp_trapezoid_system(4, 10, fake, 0.1, fake, fake, fake, fake, None, fake,
                                       None) == -9


def test_plan_btri_levels_shrink_to_one_chain():
    for nb in (2, 7, 100, 65537):
        plan = pf.pf_plan(_mat(nb=nb))
        assert plan[0][1] == nb
        for (k, n, p), nxt in zip(plan, plan[1:]):
            assert k == pf.PF_BTRI and 2 <= p <= (n + 1) // 2
            assert nxt[1] == p - 1          # reduced matrix has p-1 blocks
        assert plan[-1][2] == 1


def test_plan_finest_chain_lengths():
    """Level-0 partitions of the planner: 16 blocks for m <= 8 and for the
    FP64 bidiagonal-plus-corner form with m = 16 (its matrix-core kernel
    inverts four blocks at a time), 4 for other m >= 16 and for FP32 factors
    of that form."""
    def p0(kind, m, nb, prec=pf.PF_FP64):
        return pf.pf_plan(_mat(kind, m, nb), pf.make_opts(prec=prec))[0][2]
    assert p0(pf.PF_BTRI, 8, 65537) == (65537 + 1) // 17
    assert p0(pf.PF_BABD, 16, 262145) == (262145 - 1) // 17
    # FP32 factors of this form: 4 blocks in the table, doubled to 8 because
    # 262144 / 9 partitions leave room (the chain rule below)
    assert p0(pf.PF_BABD, 16, 262145, pf.PF_FP32_IR) == (262145 - 1) // 9
    assert p0(pf.PF_BTRI, 16, 65537) == (65537 + 1) // 5
    assert p0(pf.PF_BABD, 12, 262145) == (262145 - 1) // 17    # padded to 16


def test_plan_finest_chain_grows_with_spare_partitions():
    """The finest level keeps the table's chain until it has partitions to
    spare: the chain doubles, up to 64 blocks, while at least 16384
    partitions remain.  Scalar systems and an explicit block_rows keep
    theirs."""
    n20 = 1 << 20

    def p0(kind, m, nb, **kw):
        return pf.pf_plan(_mat(kind, m, nb), pf.make_opts(**kw))[0][2]
    # m = 32: table 4; 2^20 blocks: 8, 16, 32 (2^20 / 33 >= 16384), not 64
    assert p0(pf.PF_BTRI, 32, 65537) == 65538 // 5
    assert p0(pf.PF_BTRI, 32, n20) == (n20 + 1) // 33
    # m = 8: table 16; 2^20 blocks: 32, not 64 (2^20 / 65 < 16384)
    assert p0(pf.PF_BTRI, 8, n20) == (n20 + 1) // 33
    # the bidiagonal-plus-corner form (table 16 in FP64): 32
    assert p0(pf.PF_BABD, 16, n20 + 1) == n20 // 33
    # an explicit chain length, and scalar systems, are kept
    assert p0(pf.PF_BTRI, 32, n20, block_rows=4) == (n20 + 1) // 5
    assert p0(pf.PF_BTRI, 1, 1 << 24) == pf.pf_plan(
        _mat(pf.PF_BTRI, 1, 1 << 24), pf.make_opts(block_rows=16))[0][2]


def test_plan_reduced_chain_lengths():
    """Reduced levels of block tridiagonal matrices: 3 blocks per partition,
    8 for scalar tridiagonal matrices (their chains run out of LDS); a
    reduced level of at most 6 blocks (17 for scalar tridiagonal matrices)
    is one chain."""
    for m, L, tail in ((1, 8, 17), (8, 3, 6)):
        plan = pf.pf_plan(_mat(pf.PF_BTRI, m, 1 << 20))
        for k, n, p in plan[1:]:
            want = 1 if n <= tail else min(max((n + 1) // (L + 1), 2), (n + 1) // 2)
            assert p == want, (m, n, p, want)
        assert plan[-1][2] == 1
    assert len(pf.pf_plan(_mat(pf.PF_BTRI, 1, 1 << 24))) == 7


def test_plan_reduced_size_depends_only_on_p():
    """The block size of T_p depends only on p, not on n (eq. (redmatr))."""
    for nb in (1000, 5000, 65537):
        plan = pf.pf_plan(_mat(nb=nb), pf.make_opts(partitions=256))
        assert plan[0][2] == 256 and plan[1][1] == 255


def test_plan_babd_levels():
    for nb in (2, 3, 5, 262145):
        plan = pf.pf_plan(_mat(pf.PF_BABD, 16, nb))
        for (k, n, p), nxt in zip(plan, plan[1:]):
            assert k == pf.PF_BABD and 1 <= p <= (n - 1) // 2
            assert nxt[1] == p + 1          # reduced matrix has p+1 blocks
        assert plan[-1] == (pf.PF_BTRI, 2, 1)


def test_factor_bytes_grow_with_size_and_precision():
    A = _mat(nb=65537)
    b64 = pf.pf_factor_bytes(A, pf.make_opts())
    b32 = pf.pf_factor_bytes(A, pf.make_opts(prec=pf.PF_FP32_IR))
    assert b64 > 4 * 65537 * 64 * 8 * 0.99
    assert b32 < b64
    assert pf.pf_factor_bytes(_mat(nb=1000)) < b64


def test_allocator_callback_and_hip_errors():
    """Factor memory goes through the caller's allocator: a NULL from it is
    PF_ENOMEM (no device work is queued: the sizes come from a host-side
    counting pass, at least pf_factor_bytes).  Setting only one of the two
    functions is an argument error; NULL, NULL restores the default."""
    lib = pf.load()
    A = _mat(m=8, nb=1000)
    h = ctypes.c_void_p()
    asked = []
    try:
        pf.pf_set_allocator(lambda n, st: (asked.append(n), 0)[1], lambda p, n, st: None)
        assert lib.pf_factor(ctypes.byref(A), None, None, ctypes.byref(h)) == pf.PF_ENOMEM
        assert len(asked) == 1 and asked[0] >= pf.pf_factor_bytes(A)
        assert pf.pf_last_hip_error() == 2          # hipErrorOutOfMemory
    finally:
        pf.pf_set_allocator()
    only_alloc = pf.ALLOC_FN(lambda n, s, c: None)
    only_free = pf.FREE_FN(lambda p, n, s, c: None)
    assert lib.pf_set_allocator(only_alloc, pf.FREE_FN(), None) == -2
    assert lib.pf_set_allocator(pf.ALLOC_FN(), only_free, None) == -1
    assert lib.pf_set_allocator(pf.ALLOC_FN(), pf.FREE_FN(), None) == 0


def test_hip_error_is_reported_not_enomem():
    """A device allocation that fails for a reason other than memory (here:
    no HIP device in the process) returns PF_EHIP, and pf_last_hip_error
    gives the HIP code (hipErrorNoDevice = 100)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("needs a process without a HIP device")
    lib = pf.load()
    A = _mat(m=8, nb=1000)
    h = ctypes.c_void_p()
    assert lib.pf_factor(ctypes.byref(A), None, None, ctypes.byref(h)) == pf.PF_EHIP
    assert pf.pf_last_hip_error() == 100


def test_solve_batch_existing_factor_checked():
    """pf_solve_batch takes existing factors in: argument checks run first
    (a bad matrix is still -2 with a factors array present)."""
    lib = pf.load()
    bad = (pf.pf_matrix * 1)(_mat(nb=1))
    nr = (ctypes.c_int32 * 1)(1)
    vp = (ctypes.c_void_p * 1)(256)
    ld = (ctypes.c_int64 * 1)(8)
    fac = (ctypes.c_void_p * 1)()
    assert lib.pf_solve_batch(1, bad, None, nr, vp, ld, vp, ld, None, fac, None) == -2
