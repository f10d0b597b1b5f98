"""Seeded synthetic inputs for the structured systems A x = f.

This module only draws random numbers and lays them out in the structure of
the workloads (ODE discretizations and random block systems).  It holds no
part of the solver's arithmetic; the solver (HIP library) and the test
oracle both consume what it returns.

Block arrays are numpy ``float64`` of shape ``(count, m, m)`` indexed
``[k, i, j]`` (entry (i, j) of block k).  ``to_device_blocks`` turns them into
the library's column-major block layout.

Structures (the paper's Sec. 2 and Sec. 3):
  * BTRI (block tridiagonal, eq. (parpart) with one-block separators):
    ``D[k] = A(k,k)``, ``Lo[j] = A(j+1,j)``, ``Up[j] = A(j,j+1)``;
  * BABD (lower block bidiagonal plus top-right corner, the form after
    eq. (redmatr1)): ``D[k] = A(k,k)``, ``Lo[j] = A(j+1,j)``, ``C = A(0,nb-1)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 9123678


def seed_for(config: int, replicate: int = 0) -> int:
    return SEED_BASE + 100 * config + replicate


@dataclasses.dataclass
class System:
    kind: str                 # "btri" or "babd"
    D: np.ndarray             # (nb, m, m)
    Lo: np.ndarray            # (nb-1, m, m)
    Up: Optional[np.ndarray]  # (nb-1, m, m) for btri, None for babd
    C: Optional[np.ndarray]   # (m, m) corner for babd, None for btri
    f: np.ndarray             # (n,) or (n, nrhs)
    x_true: Optional[np.ndarray] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.D.shape[1])

    @property
    def nb(self) -> int:
        return int(self.D.shape[0])

    @property
    def n(self) -> int:
        return self.m * self.nb


# ---------------------------------------------------------------------------
# Input construction helpers (structure only).

def btri_apply(D, Lo, Up, x):
    """A x for a BTRI matrix -- used only to build manufactured right-hand
    sides f = A x_true, as the workload recipes prescribe."""
    nb, m, _ = D.shape
    X = x.reshape(nb, m, -1)
    Y = np.einsum("kij,kjr->kir", D, X)
    if nb > 1:
        Y[1:] += np.einsum("kij,kjr->kir", Lo, X[:-1])
        Y[:-1] += np.einsum("kij,kjr->kir", Up, X[1:])
    return Y.reshape(x.shape)


def babd_apply(D, Lo, C, x):
    nb, m, _ = D.shape
    X = x.reshape(nb, m, -1)
    Y = np.einsum("kij,kjr->kir", D, X)
    if nb > 1:
        Y[1:] += np.einsum("kij,kjr->kir", Lo, X[:-1])
    Y[0] += C @ X[nb - 1]
    return Y.reshape(x.shape)


def _rhs_shape(n, nrhs):
    return (n,) if nrhs is None else (n, nrhs)


# ---------------------------------------------------------------------------
# Workload 1: scalar tridiagonal, strictly diagonally dominant.

def scalar_tridiagonal(n: int = 4096, seed: int = seed_for(1), nrhs=None) -> System:
    """Sub/super diagonals U[-1,1], diagonal 4+U[0,1]; x_true ~ N(0,1);
    f = A x_true (m = 1 block tridiagonal)."""
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-1.0, 1.0, n - 1)
    up = rng.uniform(-1.0, 1.0, n - 1)
    d = 4.0 + rng.uniform(0.0, 1.0, n)
    x = rng.standard_normal(_rhs_shape(n, nrhs))
    D, Lo, Up = d.reshape(n, 1, 1), lo.reshape(n - 1, 1, 1), up.reshape(n - 1, 1, 1)
    f = btri_apply(D, Lo, Up, x)
    return System("btri", D, Lo, Up, None, f, x, {"workload": "scalar_tridiagonal", "n": n,
                                                 "seed": seed})


def poisson(n: int, nrhs=None) -> System:
    """Discrete 1-D Poisson matrix tridiag(-1, 2, -1) with f = 1."""
    D = np.full((n, 1, 1), 2.0)
    Lo = np.full((n - 1, 1, 1), -1.0)
    Up = np.full((n - 1, 1, 1), -1.0)
    f = np.ones(_rhs_shape(n, nrhs))
    return System("btri", D, Lo, Up, None, f, None, {"workload": "poisson", "n": n})


# ---------------------------------------------------------------------------
# Workloads 2 and 3: trapezoidal discretization of y' = M(t) y + q(t) on [0,1].

def _ode_coeffs(rng, m):
    """M(t) = M0 + t M1, entries N(0, 1/m) (variance 1/m), M0 shifted by -2I."""
    s = 1.0 / math.sqrt(m)
    M0 = rng.standard_normal((m, m)) * s - 2.0 * np.eye(m)
    M1 = rng.standard_normal((m, m)) * s
    return M0, M1


def _trapezoid_steps(M0, M1, N):
    """Step n (t_n = n h, h = 1/N): S_n y_n + R_n y_{n+1} = (h/2)(q_n + q_{n+1})
    with S_n = -(I + (h/2) M(t_n)) and R_n = I - (h/2) M(t_{n+1})."""
    m = M0.shape[0]
    h = 1.0 / N
    t = np.arange(N + 1, dtype=np.float64) * h
    I = np.eye(m)
    Mt = M0[None] + t[:, None, None] * M1[None]      # (N+1, m, m)
    S = -(I[None] + 0.5 * h * Mt[:-1])
    R = I[None] - 0.5 * h * Mt[1:]
    return S, R, h


def trapezoid_bvp_btri(N: int = 65536, m: int = 8, seed: int = seed_for(2),
                       nrhs=None) -> System:
    """Separated boundary conditions: components 0..m/2-1 fixed at t=0,
    components m/2..m-1 fixed at t=1 (values N(0,1)); q ~ N(0,1) per grid
    point and component.  The N trapezoid steps plus the two boundary
    conditions are regrouped into N+1 block rows of m rows:
      row 0 = [BC at t=0 ; lower half of step 0],
      row k = [upper half of step k-1 ; lower half of step k],
      row N = [upper half of step N-1 ; BC at t=1],
    which makes the matrix block tridiagonal with well-conditioned diagonal
    blocks."""
    rng = np.random.default_rng(seed)
    M0, M1 = _ode_coeffs(rng, m)
    S, R, h = _trapezoid_steps(M0, M1, N)
    a = m // 2
    nb = N + 1
    shape_q = (N + 1, m) if nrhs is None else (N + 1, m, nrhs)
    q = rng.standard_normal(shape_q)
    bca = rng.standard_normal((a,) if nrhs is None else (a, nrhs))
    bcb = rng.standard_normal((m - a,) if nrhs is None else (m - a, nrhs))
    rhs = 0.5 * h * (q[:-1] + q[1:])                  # (N, m[, nrhs])

    D = np.empty((nb, m, m))
    Lo = np.zeros((nb - 1, m, m))
    Up = np.zeros((nb - 1, m, m))
    Ba = np.zeros((a, m)); Ba[:, :a] = np.eye(a)
    Bb = np.zeros((m - a, m)); Bb[:, a:] = np.eye(m - a)
    D[0, :a] = Ba
    D[0, a:] = S[0, a:]
    D[1:N, :a] = R[0:N - 1, :a]
    D[1:N, a:] = S[1:N, a:]
    D[N, :a] = R[N - 1, :a]
    D[N, a:] = Bb
    Lo[:, :a] = S[:, :a]          # A(k, k-1) = upper half of step k-1
    Up[:, a:] = R[:, a:]          # A(k, k+1) = lower half of step k
    f = np.empty((nb, m) + (() if nrhs is None else (nrhs,)))
    f[0, :a] = bca
    f[0, a:] = rhs[0, a:]
    f[1:N, :a] = rhs[0:N - 1, :a]
    f[1:N, a:] = rhs[1:N, a:]
    f[N, :a] = rhs[N - 1, :a]
    f[N, a:] = bcb
    f = f.reshape((nb * m,) + (() if nrhs is None else (nrhs,)))
    return System("btri", D, Lo, Up, None, f, None,
                  {"workload": "trapezoid_bvp_btri", "N": N, "m": m, "seed": seed})


def trapezoid_babd(N: int = 262144, m: int = 16, seed: int = seed_for(3),
                   nrhs=None, q_zero: bool = True) -> System:
    """Non-separated boundary conditions B0 y(0) + B1 y(1) = beta with
    B0, B1 = I + N(0,1/m) and beta ~ N(0,1); y' = M(t) y (q = 0 unless
    q_zero is False).  Block row 0 = [B0, 0, ..., 0, B1]; block row k+1 =
    [.., S_k, R_k, ..]: D[0] = B0, D[k+1] = R_k, Lo[k] = S_k, C = B1,
    nb = N + 1 unknown blocks."""
    rng = np.random.default_rng(seed)
    M0, M1 = _ode_coeffs(rng, m)
    S, R, h = _trapezoid_steps(M0, M1, N)
    s = 1.0 / math.sqrt(m)
    B0 = np.eye(m) + rng.standard_normal((m, m)) * s
    B1 = np.eye(m) + rng.standard_normal((m, m)) * s
    nb = N + 1
    D = np.empty((nb, m, m))
    D[0] = B0
    D[1:] = R
    Lo = np.ascontiguousarray(S)
    shp = (m,) if nrhs is None else (m, nrhs)
    beta = rng.standard_normal(shp)
    f = np.zeros((nb,) + shp)
    f[0] = beta
    if not q_zero:
        qs = (N + 1, m) if nrhs is None else (N + 1, m, nrhs)
        q = rng.standard_normal(qs)
        f[1:] = 0.5 * h * (q[:-1] + q[1:])
    f = f.reshape((nb * m,) + (() if nrhs is None else (nrhs,)))
    return System("babd", D, Lo, None, B1, f, None,
                  {"workload": "trapezoid_babd", "N": N, "m": m, "seed": seed})


def ivp_lower_bidiagonal(N: int, m: int, seed: int, nrhs=None) -> System:
    """The discrete IVP of Sec. 3, eq. (My): a BABD with B0 = I and no corner
    (B1 = 0): y_0 given, then N trapezoid steps of y' = M(t) y + q(t)."""
    rng = np.random.default_rng(seed)
    M0, M1 = _ode_coeffs(rng, m)
    S, R, h = _trapezoid_steps(M0, M1, N)
    nb = N + 1
    D = np.empty((nb, m, m))
    D[0] = np.eye(m)
    D[1:] = R
    shp = (m,) if nrhs is None else (m, nrhs)
    f = np.zeros((nb,) + shp)
    f[0] = rng.standard_normal(shp)
    qs = (N + 1, m) if nrhs is None else (N + 1, m, nrhs)
    q = rng.standard_normal(qs)
    f[1:] = 0.5 * h * (q[:-1] + q[1:])
    f = f.reshape((nb * m,) + (() if nrhs is None else (nrhs,)))
    return System("babd", D, np.ascontiguousarray(S), None, np.zeros((m, m)), f, None,
                  {"workload": "ivp_lower_bidiagonal", "N": N, "m": m, "seed": seed})


def ivp_problem(m: int, p: int, N: int, seed: int, t0: float = 0.0, T: float = 1.0):
    """A linear IVP y' = L y + g(t), y(t0) = y0 on [t0, T] for the time-parallel
    driver of Sec. 3, sampled on the grid of p*N steps: L = -I + a skew part
    + N(0, 0.3/m) (eigenvalues in the left half-plane, moderate stiffness), g
    a few random sinusoids per component, y0 ~ N(0, 1).  Returns (L (m, m),
    g (p*N+1, m), y0 (m,), t0, T)."""
    rng = np.random.default_rng(seed)
    K = rng.standard_normal((m, m))
    L = -np.eye(m) + 2.0 * (K - K.T) / math.sqrt(m) + rng.standard_normal((m, m)) * (0.3 / m)
    t = t0 + (T - t0) * np.arange(p * N + 1) / (p * N)
    amp = rng.standard_normal((3, m))
    freq = rng.uniform(0.5, 6.0, (3, m))
    phase = rng.uniform(0.0, 2 * math.pi, (3, m))
    g = sum(amp[k] * np.sin(freq[k] * t[:, None] + phase[k]) for k in range(3))
    y0 = rng.standard_normal(m)
    return L, np.ascontiguousarray(g), y0, t0, T


# ---------------------------------------------------------------------------
# Workloads 4 and 5: random block tridiagonal systems.

def random_btri(nb: int, m: int, seed: int, nrhs=None, manufactured: bool = True) -> System:
    """Diagonal blocks 4I + N(0,1/m), off-diagonal blocks N(0,1/m)."""
    rng = np.random.default_rng(seed)
    s = 1.0 / math.sqrt(m)
    D = rng.standard_normal((nb, m, m)) * s + 4.0 * np.eye(m)[None]
    Lo = rng.standard_normal((nb - 1, m, m)) * s
    Up = rng.standard_normal((nb - 1, m, m)) * s
    n = nb * m
    if manufactured:
        x = rng.standard_normal(_rhs_shape(n, nrhs))
        f = btri_apply(D, Lo, Up, x)
    else:
        x = None
        f = rng.standard_normal(_rhs_shape(n, nrhs))
    return System("btri", D, Lo, Up, None, f, x,
                  {"workload": "random_btri", "nb": nb, "m": m, "seed": seed})


def random_babd(nb: int, m: int, seed: int, nrhs=None) -> System:
    """A BABD with well-conditioned random blocks (for small parity cases)."""
    rng = np.random.default_rng(seed)
    s = 1.0 / math.sqrt(m)
    D = rng.standard_normal((nb, m, m)) * s + 3.0 * np.eye(m)[None]
    Lo = rng.standard_normal((nb - 1, m, m)) * s
    C = rng.standard_normal((m, m)) * s
    n = nb * m
    x = rng.standard_normal(_rhs_shape(n, nrhs))
    f = babd_apply(D, Lo, C, x)
    return System("babd", D, Lo, None, C, f, x,
                  {"workload": "random_babd", "nb": nb, "m": m, "seed": seed})


def _failing_block(rng, m, how):
    """A diagonal block the local elimination cannot pivot on: all zeros
    ("zero"), or U diag(1, .., 1, 1e-15) V^T with random orthogonal U, V
    ("ill": condition 1e15)."""
    if how == "zero":
        return np.zeros((m, m))
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    sv = np.ones(m)
    sv[-1] = 1e-15
    return (U * sv) @ V.T


def btri_failing_pivots(nb: int, m: int, seed: int, rows, how: str = "zero",
                        nrhs=None) -> System:
    """random_btri's law with the diagonal blocks of `rows` replaced by
    failing blocks and the couplings into them from the row above removed
    (A(k, k-1) = 0), so that a partition's elimination meets them as its
    pivot blocks unchanged; the matrix as a whole stays regular (row k
    reaches x_{k+1} through A(k, k+1)).  Manufactured solution."""
    rng = np.random.default_rng(seed)
    s = 1.0 / math.sqrt(m)
    D = rng.standard_normal((nb, m, m)) * s + 4.0 * np.eye(m)[None]
    Lo = rng.standard_normal((nb - 1, m, m)) * s
    Up = rng.standard_normal((nb - 1, m, m)) * s
    for k in rows:
        D[k] = _failing_block(rng, m, how)
        if k > 0:
            Lo[k - 1] = 0.0
    x = rng.standard_normal(_rhs_shape(nb * m, nrhs))
    f = btri_apply(D, Lo, Up, x)
    return System("btri", D, Lo, Up, None, f, x,
                  {"workload": "btri_failing_pivots", "nb": nb, "m": m, "seed": seed,
                   "rows": list(rows), "how": how})


def babd_failing_pivots(nb: int, m: int, seed: int, rows, how: str = "zero",
                        nrhs=None) -> System:
    """random_babd's law with the diagonal blocks of `rows` (interior block
    rows) replaced by failing blocks; in this form the pivot blocks are the
    diagonal blocks themselves.  Manufactured solution."""
    rng = np.random.default_rng(seed)
    s = 0.3 / math.sqrt(m)
    # transfer maps -D[k+1]^{-1} Lo[k] near the identity: a block row that
    # cannot be pivoted on leaves a free block that the corner must still
    # fix, which it can only while the chain neither grows nor decays much
    D = rng.standard_normal((nb, m, m)) * s + 3.0 * np.eye(m)[None]
    Lo = rng.standard_normal((nb - 1, m, m)) * s - 3.0 * np.eye(m)[None]
    C = rng.standard_normal((m, m)) * s + np.eye(m)
    for k in rows:
        D[k] = _failing_block(rng, m, how)
    x = rng.standard_normal(_rhs_shape(nb * m, nrhs))
    f = babd_apply(D, Lo, C, x)
    return System("babd", D, Lo, None, C, f, x,
                  {"workload": "babd_failing_pivots", "nb": nb, "m": m, "seed": seed,
                   "rows": list(rows), "how": how})


def batch_specs(count: int = 512, seed: int = seed_for(4), m_choices=(4, 8, 16, 32),
                n_lo: int = 2 ** 8, n_hi: int = 2 ** 16, max_rhs: int = 64):
    """Shapes of the batched workload: m uniform over m_choices, the block
    count N log-uniform on [n_lo, n_hi] (continuous, then floor), nrhs
    uniform on 1..max_rhs.  Returns a list of (m, nb, nrhs, seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(rng.choice(m_choices))
        nb = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        nb = max(nb, 2)
        k = int(rng.integers(1, max_rhs + 1))
        out.append((m, nb, k, seed * 1000 + i))
    return out


def serving_stream(count: int, qps: float, seed: int = seed_for(5), m_choices=(8, 16, 32),
                   median_n: int = 2 ** 14, sigma: float = 1.0, n_min: int = 2 ** 8,
                   n_max: int = 2 ** 20, repeat_frac: float = 0.3):
    """Poisson arrivals at rate qps; m uniform over m_choices; N lognormal
    (median median_n, sigma in natural log, clamped to [n_min, n_max]); a
    fraction repeat_frac of requests re-solve a factor that is already
    resident (chosen uniformly) with a fresh right-hand side.  Returns a list
    of dicts with keys t (arrival, s), m, nb, repeat, seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / qps)
        m = int(rng.choice(m_choices))
        nb = int(math.floor(median_n * math.exp(sigma * rng.standard_normal())))
        nb = int(min(max(nb, n_min), n_max))
        rep = bool(i > 0 and rng.uniform() < repeat_frac)
        out.append({"t": t, "m": m, "nb": nb, "repeat": rep, "seed": seed * 1000 + i,
                    "pick": float(rng.uniform())})
    return out


# ---------------------------------------------------------------------------
# Layout conversion for the library: column-major m x m blocks, contiguous.

def colmajor_blocks(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).transpose(0, 2, 1))


def to_device_blocks(a: np.ndarray, device="cuda"):
    import torch
    return torch.from_numpy(colmajor_blocks(a)).to(device)


def to_device_rhs(f: np.ndarray, device="cuda"):
    """(n,) or (n, nrhs) -> column-major device buffer shaped (nrhs, n)."""
    import torch
    f2 = f[:, None] if f.ndim == 1 else f
    return torch.from_numpy(np.ascontiguousarray(f2.T)).to(device)
