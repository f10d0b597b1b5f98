"""GPU parity: the HIP partition-method solver against the CPU oracle, through
the C ABI.  Sizes span many partitions per wave, several waves and ragged
partition lengths; the full-size workloads are checked too."""
import numpy as np
import pytest

from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

from . import _gpu as G

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


# --------------------------------------------------------------------------
# scalar tridiagonal (m = 1)
@pytest.mark.parametrize("p", [16, 1, 2, 3, 7, 0, 2048])
def test_scalar_tridiagonal_4096(p):
    s = wl.scalar_tridiagonal(4096)
    _say("scalar n=4096 p", p)
    x, info, levels = G.gpu_solve(s, pf.make_opts(partitions=p))
    assert info.status == 0
    r = G.check(s, x, tag=f"p={p}")
    if p:
        assert levels[0][2] == p
    _say(r, levels)


def test_poisson_closed_form():
    n = 4096
    s = wl.poisson(n)
    x, info, _ = G.gpu_solve(s)
    i = np.arange(1, n + 1, dtype=np.float64)
    xe = i * (n + 1 - i) / 2.0
    kap = n * (n + 2) / 2
    fe = G.fwd_err(x, xe)
    _say("poisson fwd err", fe)
    assert fe <= 1e3 * kap * G.EPS
    assert G.eta(s, x) <= G.ETA_TOL


# --------------------------------------------------------------------------
# random block tridiagonal, all instantiated block sizes, ragged lengths
@pytest.mark.parametrize("m", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("nb", [2, 3, 7, 50, 1001, 4099])
def test_btri_random(m, nb):
    s = wl.random_btri(nb, m, seed=100 + m * 7 + nb)
    _say("btri m", m, "nb", nb)
    x, info, levels = G.gpu_solve(s)
    assert info.status == 0
    G.check(s, x, tag=f"m={m} nb={nb} levels={levels}")


@pytest.mark.parametrize("kind,nb", [("btri", 2), ("btri", 3), ("btri", 50), ("btri", 513),
                                     ("babd", 3), ("babd", 40)])
def test_block_size_32(kind, nb):
    s = wl.random_btri(nb, 32, seed=900 + nb) if kind == "btri" else wl.random_babd(nb, 32, seed=900 + nb)
    _say(kind, "m 32 nb", nb)
    x, info, levels = G.gpu_solve(s)
    assert info.status == 0
    G.check(s, x, tag=f"{kind} m=32 nb={nb} levels={levels}")


@pytest.mark.parametrize("flag", ["rows", "default", "wide", "segments"])
@pytest.mark.parametrize("kind,m,nb", [("btri", 2, 301), ("btri", 4, 1001), ("btri", 8, 4099),
                                       ("btri", 3, 77), ("btri", 8, 7), ("babd", 2, 40),
                                       ("babd", 4, 300), ("babd", 8, 1001), ("babd", 6, 31),
                                       ("btri", 16, 600), ("babd", 16, 300), ("btri", 12, 50),
                                       ("btri", 1, 999)])
def test_lane_mappings(kind, m, nb, flag):
    """Every factor lane mapping gives the oracle's solution: rows on every
    level; the planner's default (segments, and the matrix-core kernel at the
    finest level of FP64 block tridiagonal m = 8 matrices); wider segments at
    level 0 (m = 8: two entries per lane); segments only."""
    seed = 500 + m * 13 + nb
    s = wl.random_btri(nb, m, seed=seed) if kind == "btri" else wl.random_babd(nb, m, seed=seed)
    M = 1 << (m - 1).bit_length()
    if flag == "rows":
        opts = pf.make_opts(flags=pf.PF_FLAG_MAP_ROWS)
    elif flag == "wide":
        opts = pf.make_opts(lane_entries={8: 2, 16: 4}.get(M, 1))
    elif flag == "segments":
        opts = pf.make_opts(flags=pf.PF_FLAG_MAP_SEGMENTS)
    else:
        opts = pf.make_opts()
    _say(kind, "m", m, "nb", nb, flag)
    x, info, levels = G.gpu_solve(s, opts)
    assert info.status == 0
    G.check(s, x, tag=f"{kind} m={m} nb={nb} {flag} levels={levels}")


@pytest.mark.parametrize("nb,p", [(2, 1), (3, 1), (5, 2), (9, 3), (100, 7), (301, 0),
                                  (4099, 33), (65, 32), (1000, 499)])
@pytest.mark.parametrize("nrhs", [1, 3, 8])
def test_matrix_core_partitions(nb, p, nrhs):
    """The matrix-core factor kernel (m = 8, FP64 block tridiagonal, finest
    level) gives the oracle's solution and agrees with the segment mapping
    for every pairing of partitions in a wave: an odd count (the last wave's
    second partition shadows its first), lengths that differ by one, single
    partitions and one-block partitions; with the fused forward sweep for up
    to 8 right-hand sides."""
    import torch
    seed = 1300 + nb + 7 * p + nrhs
    s = wl.random_btri(nb, 8, seed=seed)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nb * 8, nrhs))
    A, keep = G.to_device(s)
    xs = {}
    for name, flags in (("mfma", 0), ("segments", pf.PF_FLAG_MAP_SEGMENTS)):
        F = pf.pf_factor(A, pf.make_opts(partitions=p, flags=flags))
        try:
            fd = G.rhs_to_device(f)
            x = torch.full_like(fd, np.nan)
            _say("nb", nb, "p", p, "nrhs", nrhs, name)
            info = pf.pf_factor_solve(F, fd, x)
            assert info.status == 0
            xs[name] = x.cpu().numpy().T
            G.check(s, xs[name], f=f, tag=f"{name} nb={nb} p={p} k={nrhs}")
            # the factors left behind serve pf_solve
            x2 = torch.full_like(fd, np.nan)
            assert pf.pf_solve(F, fd, x2).status == 0
            G.check(s, x2.cpu().numpy().T, f=f, tag=f"{name} solve nb={nb} p={p} k={nrhs}")
        finally:
            pf.pf_destroy(F)
    scale = np.abs(xs["segments"]).max()
    assert np.abs(xs["mfma"] - xs["segments"]).max() <= 1e-11 * scale
    del keep


@pytest.mark.parametrize("nb,p", [(2, 1), (3, 1), (9, 4), (100, 0), (1001, 0), (4099, 0),
                                  (600, 299), (257, 5)])
@pytest.mark.parametrize("m", [32, 27])
def test_matrix_core_32(nb, p, m):
    """The m = 32 matrix-core factor kernel (FP64 block tridiagonal, every
    level, including the reduced levels whose diagonal is a sum of two
    arrays) gives the oracle's solution and agrees with the row mapping;
    padded block sizes (m = 27) included."""
    import torch
    seed = 1500 + nb + 3 * p + m
    s = wl.random_btri(nb, m, seed=seed)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nb * m, 3))
    A, keep = G.to_device(s)
    xs = {}
    for name, flags in (("mfma", 0), ("rows", pf.PF_FLAG_MAP_ROWS)):
        F = pf.pf_factor(A, pf.make_opts(partitions=p, flags=flags))
        try:
            fd = G.rhs_to_device(f)
            x = torch.full_like(fd, np.nan)
            _say("m", m, "nb", nb, "p", p, name)
            info = pf.pf_solve(F, fd, x)
            assert info.status == 0
            xs[name] = x.cpu().numpy().T
            G.check(s, xs[name], f=f, tag=f"{name} m={m} nb={nb} p={p}")
        finally:
            pf.pf_destroy(F)
    scale = np.abs(xs["rows"]).max()
    assert np.abs(xs["mfma"] - xs["rows"]).max() <= 1e-11 * scale
    del keep


@pytest.mark.parametrize("nb,p", [(2, 1), (3, 1), (9, 4), (100, 0), (1001, 0), (4099, 0),
                                  (600, 299), (257, 5)])
@pytest.mark.parametrize("m,nrhs", [(16, 1), (16, 20), (11, 3)])
def test_matrix_core_16(nb, p, m, nrhs):
    """The m = 16 block tridiagonal matrix-core factor kernel (FP64, every
    level, the m = 32 kernel's scheme with one tile per product and four
    entries per lane in the inversion) gives the oracle's solution and
    agrees with the segment mapping; padded blocks (m = 11) and pf_factor_solve
    included."""
    import torch
    seed = 1900 + nb + 3 * p + m + nrhs
    s = wl.random_btri(nb, m, seed=seed)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nb * m, nrhs))
    A, keep = G.to_device(s)
    xs = {}
    for name, flags in (("mfma", 0), ("segments", pf.PF_FLAG_MAP_SEGMENTS)):
        F = pf.pf_factor(A, pf.make_opts(partitions=p, flags=flags))
        try:
            fd = G.rhs_to_device(f)
            x = torch.full_like(fd, np.nan)
            _say("btri m", m, "nb", nb, "p", p, "nrhs", nrhs, name)
            info = pf.pf_solve(F, fd, x)
            assert info.status == 0
            xs[name] = x.cpu().numpy().T
            G.check(s, xs[name], f=f, tag=f"{name} btri m={m} nb={nb} p={p}")
            x2 = torch.full_like(fd, np.nan)
            assert pf.pf_factor_solve(F, fd, x2).status == 0
            G.check(s, x2.cpu().numpy().T, f=f, tag=f"{name} factor_solve m={m} nb={nb} p={p}")
        finally:
            pf.pf_destroy(F)
    scale = np.abs(xs["segments"]).max()
    assert np.abs(xs["mfma"] - xs["segments"]).max() <= 1e-11 * scale
    del keep


def test_singular_pivot_btri16():
    """An exactly singular first pivot block is reported by the m = 16 block
    tridiagonal matrix-core kernel with its level and block."""
    s = wl.random_btri(64, 16, seed=6)
    s.D[0] = 0.0
    s.Up[0] = 0.0
    x, info, _ = G.gpu_solve(s, pf.make_opts(partitions=4))
    assert info.status == pf.PF_ESINGULAR
    assert info.bad_level == 0 and info.bad_block == 0


@pytest.mark.parametrize("nb,p", [(3, 1), (5, 2), (9, 4), (40, 3), (41, 3), (300, 7), (1000, 0),
                                  (4097, 0), (1001, 500)])
@pytest.mark.parametrize("m,nrhs", [(16, 1), (16, 16), (12, 5), (16, 17)])
def test_matrix_core_babd16(nb, p, m, nrhs):
    """The m = 16 matrix-core factor kernel of the bidiagonal-plus-corner form
    (FP64, every level: four pivot blocks inverted together, the chain on the
    matrix cores) gives the oracle's solution and agrees with the segment
    mapping: partitions of one to thirteen blocks (groups of four with ragged
    tails), the fused forward sweep for 1..16 right-hand sides, 17 (no
    fusion), padded blocks (m = 12), and the factors left for pf_solve."""
    import torch
    seed = 1700 + nb + 5 * p + m + nrhs
    s = wl.random_babd(nb, m, seed=seed)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nb * m, nrhs))
    A, keep = G.to_device(s)
    xs = {}
    for name, flags in (("mfma", 0), ("segments", pf.PF_FLAG_MAP_SEGMENTS)):
        F = pf.pf_factor(A, pf.make_opts(partitions=p, flags=flags))
        try:
            fd = G.rhs_to_device(f)
            x = torch.full_like(fd, np.nan)
            _say("babd m", m, "nb", nb, "p", p, "nrhs", nrhs, name)
            info = pf.pf_factor_solve(F, fd, x)
            assert info.status == 0
            xs[name] = x.cpu().numpy().T
            G.check(s, xs[name], f=f, tag=f"{name} babd m={m} nb={nb} p={p} k={nrhs}")
            x2 = torch.full_like(fd, np.nan)
            assert pf.pf_solve(F, fd, x2).status == 0
            G.check(s, x2.cpu().numpy().T, f=f, tag=f"{name} solve babd m={m} nb={nb} p={p}")
        finally:
            pf.pf_destroy(F)
    scale = np.abs(xs["segments"]).max()
    assert np.abs(xs["mfma"] - xs["segments"]).max() <= 1e-11 * scale
    del keep


@pytest.mark.parametrize("flags", [0, pf.PF_FLAG_MAP_SEGMENTS])
def test_singular_pivot_babd16(flags):
    """An exactly singular pivot block inside a partition of the m = 16
    bidiagonal-plus-corner form is reported with its level and the first such
    block, by the matrix-core kernel (blocks inverted in groups of four) as by
    the segment kernel.  Partitions of nine blocks: separators 0, 10, .., 40."""
    s = wl.random_babd(41, 16, seed=9)
    s.D[23] = 0.0
    s.D[17] = 0.0
    x, info, _ = G.gpu_solve(s, pf.make_opts(partitions=4, flags=flags))
    assert info.status == pf.PF_ESINGULAR
    assert info.bad_level == 0 and info.bad_block == 17


@pytest.mark.parametrize("kind,m,nb,nrhs,prec", [
    ("btri", 8, 4099, 1, "fp64"), ("btri", 8, 1001, 3, "fp64"), ("btri", 8, 300, 8, "fp64"),
    ("btri", 8, 300, 9, "fp64"), ("btri", 4, 2049, 1, "fp64"), ("btri", 3, 700, 2, "fp64"),
    ("btri", 2, 513, 2, "fp64"), ("btri", 16, 200, 1, "fp64"), ("btri", 1, 4096, 1, "fp64"),
    ("babd", 8, 1001, 1, "fp64"), ("babd", 4, 300, 4, "fp64"), ("babd", 6, 77, 1, "fp64"),
    ("btri", 8, 2049, 1, "fp32ir"), ("babd", 8, 1001, 2, "fp32ir")])
def test_factor_solve(kind, m, nb, nrhs, prec):
    """pf_factor_solve (refactor + solve, fused per level where it applies)
    gives the oracle's solution, leaves factors that pf_solve can reuse, and
    agrees with pf_refactor + pf_solve."""
    import torch
    seed = 700 + m * 11 + nb + nrhs
    s = wl.random_btri(nb, m, seed=seed) if kind == "btri" else wl.random_babd(nb, m, seed=seed)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nb * m, nrhs))
    A, keep = G.to_device(s)
    opts = pf.make_opts(prec=pf.PF_FP32_IR if prec == "fp32ir" else pf.PF_FP64)
    F = pf.pf_factor(A, opts)
    try:
        fd = G.rhs_to_device(f)
        x1 = torch.full_like(fd, np.nan)
        x2 = torch.full_like(fd, np.nan)
        _say(kind, m, nb, nrhs, prec)
        info = pf.pf_factor_solve(F, fd, x1)
        assert info.status == 0
        G.check(s, x1.cpu().numpy().T, f=f, tag=f"factor_solve {kind} m={m} nb={nb} k={nrhs}")
        pf.pf_refactor(F)
        info = pf.pf_solve(F, fd, x2)
        assert info.status == 0
        a, b = x1.cpu().numpy(), x2.cpu().numpy()
        assert np.abs(a - b).max() <= (1e-13 if prec == "fp64" else 1e-10) * np.abs(b).max()
        f3 = rng.standard_normal((nb * m, 1))       # the stored factors serve a new solve
        f3d = G.rhs_to_device(f3)
        x3 = torch.empty_like(f3d)
        pf.pf_factor_solve(F, f3d, x3, nrhs=0)      # nrhs = 0: refactor only
        info = pf.pf_solve(F, f3d, x3)
        G.check(s, x3.cpu().numpy().T, f=f3, tag="after factor_solve")
    finally:
        pf.pf_destroy(F)
    del keep


@pytest.mark.parametrize("m", [4, 8])
@pytest.mark.parametrize("nrhs", [2, 5, 9])
def test_btri_multi_rhs(m, nrhs):
    s = wl.random_btri(777, m, seed=300 + nrhs, nrhs=nrhs)
    x, info, _ = G.gpu_solve(s)
    assert info.status == 0
    G.check(s, x, tag=f"m={m} nrhs={nrhs}")


@pytest.mark.parametrize("m", [8])
@pytest.mark.parametrize("p", [1, 2, 5, 64, 256, 0])
def test_p_invariance(m, p):
    s = wl.random_btri(1025, m, seed=41)
    x, info, _ = G.gpu_solve(s, pf.make_opts(partitions=p))
    x0 = G.oracle_solve(s)
    assert G.fwd_err(x, x0) <= 1e-12
    G.check(s, x, tag=f"p={p}")


@pytest.mark.parametrize("m,kind", [(8, "btri"), (16, "btri"), (32, "btri"), (16, "babd")])
@pytest.mark.parametrize("br", [32, 64])
def test_long_finest_chains(m, kind, br):
    """Chains of 32 and 64 blocks at the finest level (the planner's choice
    for systems with partitions to spare) on the matrix-core kernels, against
    the oracle."""
    import torch
    nb = 2000 if m < 32 else 1200
    s = wl.random_btri(nb, m, seed=43 + m) if kind == "btri" else wl.random_babd(nb, m, seed=43 + m)
    x, info, levels = G.gpu_solve(s, pf.make_opts(block_rows=br))
    assert info.status == 0
    G.check(s, x, tag=f"{kind} m={m} block_rows={br} levels={levels[:2]}")
    # the fused factor-and-solve call (its finest level sweeps forward in the
    # factor kernel where it can)
    A, keep = G.to_device(s)
    F = pf.pf_factor(A, pf.make_opts(block_rows=br))
    try:
        fd = G.rhs_to_device(s.f)
        xd = torch.full_like(fd, np.nan)
        assert pf.pf_factor_solve(F, fd, xd).status == 0
        torch.cuda.synchronize()
    finally:
        pf.pf_destroy(F)
    del keep
    G.check(s, xd.cpu().numpy().T.reshape(x.shape), tag=f"fused {kind} m={m} block_rows={br}")


@pytest.mark.parametrize("br", [1, 2, 3, 5, 16, 40])
def test_block_rows_invariance(br):
    s = wl.random_btri(3001, 4, seed=42)
    x, info, levels = G.gpu_solve(s, pf.make_opts(block_rows=br))
    G.check(s, x, tag=f"block_rows={br} levels={levels}")


@pytest.mark.parametrize("m", [3, 5, 6, 12])
def test_btri_padded_block_sizes(m):
    s = wl.random_btri(333, m, seed=500 + m, nrhs=2)
    x, info, _ = G.gpu_solve(s)
    assert info.status == 0
    G.check(s, x, tag=f"m={m}")


# --------------------------------------------------------------------------
# ODE-BVP workloads
def test_trapezoid_btri_small():
    s = wl.trapezoid_bvp_btri(N=4096, m=8, seed=wl.seed_for(2, 1))
    x, info, _ = G.gpu_solve(s, pf.make_opts(partitions=256))
    _say(G.check(s, x, tag="trapezoid N=4096"))


def test_trapezoid_btri_full():
    """Block tridiagonal trapezoid BVP, N = 65536 steps, m = 8, 256 partitions."""
    s = wl.trapezoid_bvp_btri(N=65536, m=8)
    kap = G.kappa(s)
    for p in (256, 0):
        x, info, levels = G.gpu_solve(s, pf.make_opts(partitions=p))
        assert info.status == 0
        _say("trapezoid full p", p, levels, G.check(s, x, kap=kap, tag=f"full p={p}"))


@pytest.mark.parametrize("m,nb", [(1, 9), (2, 3), (4, 40), (8, 101), (16, 1000), (8, 5)])
def test_babd_random(m, nb):
    s = wl.random_babd(nb, m, seed=600 + m + nb, nrhs=2)
    x, info, levels = G.gpu_solve(s)
    assert info.status == 0
    G.check(s, x, tag=f"babd m={m} nb={nb} levels={levels}")


@pytest.mark.parametrize("p", [1, 2, 3, 100, 0])
def test_babd_trapezoid_small(p):
    s = wl.trapezoid_babd(N=4096, m=16, seed=wl.seed_for(3, 1))
    x, info, levels = G.gpu_solve(s, pf.make_opts(partitions=p))
    assert info.status == 0
    G.check(s, x, tag=f"babd N=4096 p={p}")


def test_ivp_lower_bidiagonal():
    """B1 = 0, B0 = I: the discrete IVP of Sec. 3 through the same path."""
    s = wl.ivp_lower_bidiagonal(N=20000, m=4, seed=77)
    x, info, _ = G.gpu_solve(s)
    G.check(s, x, tag="ivp")


def test_fp32_ir_babd_small():
    s = wl.trapezoid_babd(N=4096, m=16, seed=wl.seed_for(3, 2))
    x, info, _ = G.gpu_solve(s, pf.make_opts(prec=pf.PF_FP32_IR))
    _say("fp32 ir", info.as_dict())
    assert info.status == 0
    assert info.eta <= 1e-12
    G.check(s, x, tag="fp32ir")


def test_fp32_ir_btri():
    s = wl.random_btri(5000, 8, seed=88, nrhs=3)
    x, info, _ = G.gpu_solve(s, pf.make_opts(prec=pf.PF_FP32_IR))
    _say("fp32 ir btri", info.as_dict())
    assert info.status == 0
    G.check(s, x, tag="fp32ir btri")


# --------------------------------------------------------------------------
# error path: an exactly singular pivot block
@pytest.mark.parametrize("flags", [0, pf.PF_FLAG_MAP_ROWS])
def test_singular_pivot_reported(flags):
    s = wl.random_btri(64, 4, seed=5)
    s.D[0] = 0.0
    s.Up[0] = 0.0
    x, info, _ = G.gpu_solve(s, pf.make_opts(partitions=4, flags=flags))
    assert info.status == pf.PF_ESINGULAR
    assert info.bad_level == 0 and info.bad_block == 0
