"""GPU tests of the FP64 residual r = f - A x and the norms of the normwise
backward error (pf_residual: the refinement's residual and PF_FLAG_ETA's
check), against the oracle's residual and norm on the same seeded inputs.

x is random, not a solution, so r is of the size of its terms and the two
sides differ only by the rounding of their sums.  A row of r sums 3m + 1
terms at most (two block diagonals and the diagonal, or the corner, and f),
so each side is within gamma_{3m+1} (|A| |x| + |f|) of the exact value
(gamma_k = k u / (1 - k u), u = 2^-53, the standard bound for a recursive or
blocked sum of products), and the two within twice that.  The max-abs norms
of x and f are exact on both sides; ||A||_inf's row sums of 3m terms differ
by at most 2 gamma_{3m} ||A||."""
import numpy as np
import pytest

import oracle
from paper_0912_3678_amd import pf
from paper_0912_3678_amd import workloads as wl

from . import _gpu as G

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _gamma(k):
    return k * U / (1 - k * U)


def _say(*a):
    print(*a, flush=True)


def _case(kind, m, nb, k, seed, pad):
    import torch
    s = wl.random_btri(nb, m, seed=seed) if kind == "btri" else wl.random_babd(nb, m, seed=seed)
    A, keep = G.to_device(s)
    n = s.n
    rng = np.random.default_rng(seed + 1)
    f = rng.standard_normal((n, k))
    x = rng.standard_normal((n, k)) * np.exp(rng.uniform(-2, 2, size=k))   # columns of mixed size
    ld = n + pad
    dev = G.device()

    def put(a):
        t = torch.zeros((k, ld), dtype=torch.float64, device=dev)
        t[:, :n] = torch.tensor(a.T, device=dev)
        return t
    fd, xd = put(f), put(x)
    rd = torch.full((k, ld), np.nan, dtype=torch.float64, device=dev)
    norms, na = pf.pf_residual(A, fd, xd, rd, nrhs=k, ldf=ld, ldx=ld, ldr=ld)
    norms0, na0 = pf.pf_residual(A, fd, xd, None, nrhs=k, ldf=ld, ldx=ld)   # norms only
    torch.cuda.synchronize()
    r = rd[:, :n].cpu().numpy().T
    assert np.isnan(rd[:, n:].cpu().numpy()).all(), "wrote past the rows of r"
    zero = np.zeros_like(f)
    if kind == "btri":
        ro = oracle.btri_residual(s.D, s.Lo, s.Up, f, x)
        nao = oracle.btri_norminf(s.D, s.Lo, s.Up)
        # |A| |x| as minus the residual of |A| against |x| with f = 0
        ax = -oracle.btri_residual(np.abs(s.D), np.abs(s.Lo), np.abs(s.Up), zero, np.abs(x))
    else:
        ro = oracle.babd_residual(s.D, s.Lo, s.C, f, x)
        nao = oracle.babd_norminf(s.D, s.Lo, s.C)
        ax = -oracle.babd_residual(np.abs(s.D), np.abs(s.Lo), np.abs(s.C), zero, np.abs(x))
    scale = ax + np.abs(f)
    bound = 2 * _gamma(3 * m + 1) * scale
    err = np.abs(r - ro)
    tag = f"{kind} m={m} nb={nb} nrhs={k} pad={pad}"
    _say(tag, "max err / bound", float((err / bound).max()))
    assert (err <= bound).all(), f"{tag}: residual outside the rounding bound"
    # norms per column: ||r||, ||x||, ||f||
    assert np.array_equal(norms[:, 1], np.abs(x).max(0)), f"{tag}: ||x||"
    assert np.array_equal(norms[:, 2], np.abs(f).max(0)), f"{tag}: ||f||"
    assert (np.abs(norms[:, 0] - np.abs(ro).max(0)) <= bound.max(0)).all(), f"{tag}: ||r||"
    assert abs(na - nao) <= 2 * _gamma(3 * m) * nao, f"{tag}: ||A|| {na} vs {nao}"
    # the norms-only pass computes the same norms
    assert np.array_equal(norms0, norms) and na0 == na, f"{tag}: norms-only pass differs"
    del keep


# block sizes on the matrix cores (4, 8, 16, 32) and on the vector units
# (1, 3); nb = 37 leaves ragged 16-row groups for m = 4 and 8; nrhs 17 and 70
# leave ragged column tiles and a second chunk of 64 columns
@pytest.mark.parametrize("kind", ["btri", "babd"])
@pytest.mark.parametrize("m", [1, 3, 4, 8, 16, 32])
@pytest.mark.parametrize("k", [1, 17, 70])
def test_residual_matches_oracle(kind, m, k):
    _case(kind, m, 37, k, seed=6100 + 10 * m + k, pad=5 if k == 17 else 0)


@pytest.mark.parametrize("kind", ["btri", "babd"])
@pytest.mark.parametrize("m", [4, 8, 16, 32])
def test_residual_two_block_rows(kind, m):
    _case(kind, m, 2, 3, seed=6200 + m, pad=0)


@pytest.mark.parametrize("m,nb", [(8, 40000), (32, 6000)])
def test_residual_many_groups(m, nb):
    # more row groups than the grid's 4096 waves: each wave strides over several
    _case("btri", m, nb, 2, seed=6300 + m, pad=0)
