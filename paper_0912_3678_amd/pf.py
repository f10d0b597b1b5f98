"""Python binding of the C ABI in ``include/pf.h`` (ctypes; argument
marshalling only -- every step of the method runs in the HIP library).

Device buffers are torch tensors on a HIP device; streams are torch streams.
The library must be built (``paper_0912_3678_amd.build``); importing the
binding without it raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpf.so")

PF_BTRI, PF_BABD = 0, 1
PF_FP64, PF_FP32_IR = 0, 1
PF_OK, PF_ESINGULAR, PF_ENOCONV, PF_ENOMEM, PF_EHIP, PF_EUNSUPPORTED = 0, 1, 2, 3, 4, 5
PF_ETOOBIG = 6
PF_FLAG_ETA = 1
PF_FLAG_MAP_ROWS, PF_FLAG_MAP_TILES, PF_FLAG_AUTOTUNE, PF_FLAG_MAP_SEGMENTS = 2, 4, 8, 16
PF_FLAG_ENLARGE = 32

EXPORTED = [
    "pf_factor", "pf_solve", "pf_solve_batch", "pf_factor_bytes", "pf_solve_bytes_per_rhs",
    "pf_sync_status", "pf_destroy", "pf_strerror", "pf_factor_levels", "pf_factor_level",
    "pf_factor_block_size", "pf_factor_export_reduced", "pf_band_to_btri", "pf_abd_to_btri",
    "pf_ivp_trapezoid_system", "pf_ivp_solve", "pf_ivp_create", "pf_ivp_run", "pf_ivp_destroy",
    "pf_plan", "pf_refactor", "pf_profile_enable", "pf_profile_read",
    "pf_batch_create", "pf_batch_run", "pf_batch_factor", "pf_batch_destroy", "pf_factor_solve",
    "pf_autotune", "pf_autotune_clear",
    "pf_server_create", "pf_server_submit", "pf_server_poll", "pf_server_wait", "pf_server_times",
    "pf_server_release", "pf_server_stats", "pf_server_destroy",
    "pf_set_allocator", "pf_last_hip_error", "pf_factor_solve_static", "pf_batch_profile",
    "pf_server_reserve", "pf_residual",
]


class pf_matrix(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("m", ctypes.c_int32), ("nb", ctypes.c_int64),
                ("D", ctypes.c_void_p), ("Lo", ctypes.c_void_p), ("Up", ctypes.c_void_p),
                ("C", ctypes.c_void_p)]


class pf_opts(ctypes.Structure):
    _fields_ = [("partitions", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("block_rows", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("coarse_rows", ctypes.c_int32),
                ("lane_entries", ctypes.c_int32), ("tol", ctypes.c_double)]


class pf_launch_info(ctypes.Structure):
    _fields_ = [("phase", ctypes.c_int32), ("level", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("m", ctypes.c_int32), ("f32", ctypes.c_int32), ("mapping", ctypes.c_int32),
                ("rows", ctypes.c_int64), ("rhs_rows", ctypes.c_int64),
                ("workgroups", ctypes.c_int32), ("ms", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pf_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("refine_iters", ctypes.c_int32),
                ("bad_level", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("bad_block", ctypes.c_int64), ("eta", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                           ctypes.c_void_p)
_allocator = None   # the callbacks the library holds (kept alive here)


def load(path: str = LIB_PATH):
    """Load libpf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_0912_3678_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    sigs = {
        "pf_factor": (ctypes.c_int, [P(pf_matrix), P(pf_opts), vp, P(vp)]),
        "pf_solve": (ctypes.c_int, [vp, i32, vp, i64, vp, i64, vp, P(pf_info)]),
        "pf_factor_solve": (ctypes.c_int, [vp, i32, vp, i64, vp, i64, vp, P(pf_info)]),
        "pf_solve_batch": (ctypes.c_int, [i32, P(pf_matrix), P(pf_opts), P(i32), P(vp), P(i64),
                                          P(vp), P(i64), vp, P(vp), P(pf_info)]),
        "pf_factor_bytes": (ctypes.c_size_t, [P(pf_matrix), P(pf_opts)]),
        "pf_solve_bytes_per_rhs": (ctypes.c_size_t, [P(pf_matrix), P(pf_opts)]),
        "pf_sync_status": (ctypes.c_int, [vp, P(pf_info)]),
        "pf_destroy": (None, [vp]),
        "pf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "pf_factor_levels": (ctypes.c_int, [vp]),
        "pf_refactor": (ctypes.c_int, [vp, vp]),
        "pf_profile_enable": (ctypes.c_int, [vp, ctypes.c_int]),
        "pf_profile_read": (ctypes.c_int, [vp, i32, P(i32), P(i32), P(ctypes.c_float)]),
        "pf_plan": (ctypes.c_int, [P(pf_matrix), P(pf_opts), i32, P(i32), P(i64), P(i64)]),
        "pf_factor_level": (ctypes.c_int, [vp, ctypes.c_int, P(i32), P(i64), P(i64)]),
        "pf_factor_block_size": (ctypes.c_int, [vp]),
        "pf_factor_export_reduced": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
        "pf_band_to_btri": (ctypes.c_int, [i64, i32, i32, vp, i64, vp, vp, vp, vp]),
        "pf_abd_to_btri": (ctypes.c_int, [i32, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp]),
        "pf_ivp_trapezoid_system": (ctypes.c_int, [i32, i64, vp, ctypes.c_double, vp, vp, vp, vp,
                                                   vp, vp, vp]),
        "pf_ivp_solve": (ctypes.c_int, [i32, vp, ctypes.c_double, ctypes.c_double, i64, i64, vp,
                                        vp, vp, P(pf_opts), vp, P(pf_info)]),
        "pf_ivp_create": (ctypes.c_int, [i32, i64, i64, P(pf_opts), vp, P(vp)]),
        "pf_ivp_run": (ctypes.c_int, [vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp,
                                      P(pf_info)]),
        "pf_ivp_destroy": (None, [vp]),
        "pf_batch_create": (ctypes.c_int, [i32, P(pf_matrix), P(pf_opts), P(i32), P(vp), P(i64),
                                           P(vp), P(i64), vp, P(vp)]),
        "pf_batch_run": (ctypes.c_int, [vp, vp, P(pf_info)]),
        "pf_batch_factor": (ctypes.c_int, [vp, i32, P(vp)]),
        "pf_batch_profile": (ctypes.c_int, [vp, vp, i32, P(pf_launch_info), P(i32)]),
        "pf_batch_destroy": (None, [vp]),
        "pf_autotune": (ctypes.c_int, [P(pf_matrix), P(pf_opts), i32, vp, P(pf_opts),
                                       P(ctypes.c_float)]),
        "pf_autotune_clear": (None, []),
        "pf_set_allocator": (ctypes.c_int, [ALLOC_FN, FREE_FN, vp]),
        "pf_last_hip_error": (ctypes.c_int, []),
        "pf_factor_solve_static": (ctypes.c_int, [P(pf_matrix), P(pf_opts), i32, vp, i64, vp,
                                                  i64, vp, P(pf_info)]),
        "pf_residual": (ctypes.c_int, [P(pf_matrix), i32, vp, i64, vp, i64, vp, i64, vp,
                                       P(ctypes.c_double)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def pf_set_allocator(alloc=None, free=None):
    """Route the library's factor memory through Python callables:
    alloc(bytes, stream_ptr) -> device address (int, 0 when out of memory),
    free(ptr, bytes, stream_ptr).  No arguments: back to the default
    (stream-ordered hipMallocAsync)."""
    global _allocator
    lib = load()
    if alloc is None and free is None:
        rc = lib.pf_set_allocator(ALLOC_FN(), FREE_FN(), None)
        _allocator = None
    else:
        a = ALLOC_FN(lambda n, st, ctx: alloc(int(n), st or 0) or None)
        f = FREE_FN(lambda p, n, st, ctx: free(int(p), int(n), st or 0))
        rc = lib.pf_set_allocator(a, f, None)
        if rc == 0:
            _allocator = (a, f)
    if rc != 0:
        raise PFError(rc, "pf_set_allocator")


def use_torch_allocator(device=None):
    """Back the library's factor memory with PyTorch's caching allocator (on
    the stream each handle works on).  Returns the dict of live blocks
    {ptr: bytes} for inspection."""
    import torch
    dev = torch.cuda.current_device() if device is None else device
    live = {}

    def alloc(n, st):
        try:
            p = torch.cuda.caching_allocator_alloc(n, dev, int(st))
        except RuntimeError:
            return 0
        live[p] = n
        return p

    def free(p, n, st):
        live.pop(p, None)
        torch.cuda.caching_allocator_delete(p)

    pf_set_allocator(alloc, free)
    return live


def pf_last_hip_error() -> int:
    return int(load().pf_last_hip_error())


class PFError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = load().pf_strerror(code).decode()
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_matrix(kind, m, nb, D, Lo, Up=None, C=None) -> pf_matrix:
    """Device tensors (column-major blocks, FP64, contiguous) -> pf_matrix."""
    for t in (D, Lo, Up, C):
        if t is not None:
            if t.dtype.itemsize != 8 or not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError("matrix arrays must be contiguous FP64 device tensors")
    return pf_matrix(kind, m, nb, _ptr(D).value if D is not None else None,
                     _ptr(Lo).value if Lo is not None else None,
                     _ptr(Up).value if Up is not None else None,
                     _ptr(C).value if C is not None else None)


def make_opts(partitions=0, prec=PF_FP64, max_refine=0, block_rows=0, flags=0, tol=0.0,
              coarse_rows=0, lane_entries=0):
    return pf_opts(partitions, prec, max_refine, block_rows, flags, coarse_rows, lane_entries,
                   tol)


def pf_factor(A: pf_matrix, opts: pf_opts | None = None, stream=None):
    h = ctypes.c_void_p()
    rc = load().pf_factor(ctypes.byref(A), ctypes.byref(opts) if opts is not None else None,
                          _stream(stream), ctypes.byref(h))
    if rc != 0:
        raise PFError(rc, "pf_factor")
    return h


def _solve(fn, name, F, f, x, nrhs, ldf, ldx, stream, want_info):
    if nrhs is None:
        nrhs = 1 if f.dim() == 1 else f.shape[0]
    n = f.shape[-1]
    ldf = n if ldf is None else ldf
    ldx = n if ldx is None else ldx
    info = pf_info() if want_info else None
    rc = fn(F, nrhs, _ptr(f), ldf, _ptr(x), ldx, _stream(stream),
            ctypes.byref(info) if info is not None else None)
    if rc < 0 or rc in (PF_ENOMEM, PF_EHIP, PF_EUNSUPPORTED):
        raise PFError(rc, name)
    return info


def pf_solve(F, f, x, nrhs=None, ldf=None, ldx=None, stream=None, want_info=True):
    """f, x: device FP64 tensors holding n x nrhs column-major data (shape
    (nrhs, n) or (n,)).  Returns a pf_info (synchronizing) or None."""
    return _solve(load().pf_solve, "pf_solve", F, f, x, nrhs, ldf, ldx, stream, want_info)


def pf_factor_solve(F, f, x, nrhs=None, ldf=None, ldx=None, stream=None, want_info=True):
    """Refactor (the values behind the handle's matrix pointers) and solve in
    one call; arguments as pf_solve."""
    return _solve(load().pf_factor_solve, "pf_factor_solve", F, f, x, nrhs, ldf, ldx, stream,
                  want_info)


def pf_residual(A: pf_matrix, f, x, r=None, nrhs=None, ldf=None, ldx=None, ldr=None,
                stream=None):
    """r = f - A x (FP64) into r (a device tensor like f, or None) and the
    norms of eta: returns (norms per column as an (nrhs, 3) array of
    ||r||, ||x||, ||f||, ||A||)."""
    import numpy as np
    if nrhs is None:
        nrhs = 1 if f.dim() == 1 else f.shape[0]
    n = f.shape[-1]
    out = (ctypes.c_double * (3 * nrhs + 1))()
    rc = load().pf_residual(ctypes.byref(A), nrhs, _ptr(f), n if ldf is None else ldf, _ptr(x),
                            n if ldx is None else ldx, _ptr(r),
                            (n if ldr is None else ldr) if r is not None else n,
                            _stream(stream), out)
    if rc != 0:
        raise PFError(rc, "pf_residual")
    v = np.frombuffer(out, dtype=np.float64).copy()
    return v[:3 * nrhs].reshape(nrhs, 3), float(v[3 * nrhs])


def pf_factor_solve_static(A: pf_matrix, f, x, opts: pf_opts | None = None, nrhs=None,
                           ldf=None, ldx=None, stream=None, want_info=True):
    """Factor-and-solve with no device allocation (the library's static
    workspace); returns pf_info (synchronizing) or None."""
    if nrhs is None:
        nrhs = 1 if f.dim() == 1 else f.shape[0]
    n = f.shape[-1]
    info = pf_info() if want_info else None
    rc = load().pf_factor_solve_static(ctypes.byref(A),
                                       ctypes.byref(opts) if opts is not None else None, nrhs,
                                       _ptr(f), n if ldf is None else ldf, _ptr(x),
                                       n if ldx is None else ldx, _stream(stream),
                                       ctypes.byref(info) if info is not None else None)
    if rc < 0 or rc in (PF_ENOMEM, PF_EHIP, PF_EUNSUPPORTED, PF_ETOOBIG):
        raise PFError(rc, "pf_factor_solve_static")
    return info


def pf_refactor(F, stream=None):
    rc = load().pf_refactor(F, _stream(stream))
    if rc != 0:
        raise PFError(rc, "pf_refactor")


def pf_profile_enable(F, on=True):
    load().pf_profile_enable(F, 1 if on else 0)


PHASES = {0: "factor", 1: "forward", 2: "backward", 3: "factor+forward"}


def pf_profile_read(F):
    """[(phase name, level, ms)] of the latest factor/refactor and solve."""
    lib = load()
    n = 256
    ph = (ctypes.c_int32 * n)()
    lv = (ctypes.c_int32 * n)()
    ms = (ctypes.c_float * n)()
    cnt = lib.pf_profile_read(F, n, ph, lv, ms)
    if cnt < 0:
        raise PFError(cnt, "pf_profile_read")
    return [(PHASES[ph[i]], lv[i], float(ms[i])) for i in range(min(cnt, n))]


def pf_sync_status(F) -> pf_info:
    info = pf_info()
    load().pf_sync_status(F, ctypes.byref(info))
    return info


def pf_destroy(F):
    load().pf_destroy(F)


def pf_factor_bytes(A: pf_matrix, opts: pf_opts | None = None) -> int:
    return int(load().pf_factor_bytes(ctypes.byref(A), ctypes.byref(opts) if opts else None))


def pf_solve_bytes_per_rhs(A: pf_matrix, opts: pf_opts | None = None) -> int:
    return int(load().pf_solve_bytes_per_rhs(ctypes.byref(A),
                                             ctypes.byref(opts) if opts else None))


def pf_factor_levels(F):
    lib = load()
    out = []
    for l in range(lib.pf_factor_levels(F)):
        k, nb, p = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        lib.pf_factor_level(F, l, ctypes.byref(k), ctypes.byref(nb), ctypes.byref(p))
        out.append((k.value, nb.value, p.value))
    return out


def pf_plan(A: pf_matrix, opts: pf_opts | None = None):
    """Host-side level plan: list of (kind, nb, p)."""
    lib = load()
    K = (ctypes.c_int32 * 64)()
    N = (ctypes.c_int64 * 64)()
    P = (ctypes.c_int64 * 64)()
    L = lib.pf_plan(ctypes.byref(A), ctypes.byref(opts) if opts else None, 64, K, N, P)
    if L < 0:
        raise PFError(L, "pf_plan")
    return [(K[i], N[i], P[i]) for i in range(L)]


def pf_factor_block_size(F) -> int:
    return int(load().pf_factor_block_size(F))


def pf_factor_export_reduced(F, level: int):
    """Reduced matrix produced by `level` as numpy (D, Lo, Up-or-corner),
    block arrays indexed [k, i, j]."""
    import numpy as np
    kind, nb, p = pf_factor_levels(F)[level]
    M = pf_factor_block_size(F)
    nr = (p - 1) if kind == PF_BTRI else (p + 1)
    D = np.zeros((nr, M, M))
    Lo = np.zeros((max(nr - 1, 1), M, M))
    Up = np.zeros((max(nr - 1, 1) if kind == PF_BTRI else 1, M, M))
    rc = load().pf_factor_export_reduced(F, level, D.ctypes.data, Lo.ctypes.data, Up.ctypes.data)
    if rc != 0:
        raise PFError(rc, "pf_factor_export_reduced")
    tr = lambda a: np.ascontiguousarray(a.transpose(0, 2, 1))
    return tr(D), tr(Lo[:nr - 1]), (tr(Up[:nr - 1]) if kind == PF_BTRI else tr(Up)[0])


def pf_band_to_btri(n, kl, ku, ab, ldab, D, Lo, Up, stream=None):
    rc = load().pf_band_to_btri(n, kl, ku, _ptr(ab), ldab, _ptr(D), _ptr(Lo), _ptr(Up),
                                _stream(stream))
    if rc != 0:
        raise PFError(rc, "pf_band_to_btri")


def pf_abd_to_btri(m, N, qa, Ba, S, R, Bb, D, Lo, Up, stream=None):
    rc = load().pf_abd_to_btri(m, N, qa, _ptr(Ba), _ptr(S), _ptr(R), _ptr(Bb), _ptr(D),
                               _ptr(Lo), _ptr(Up), _stream(stream))
    if rc != 0:
        raise PFError(rc, "pf_abd_to_btri")


def pf_ivp_trapezoid_system(m, steps, L, h, g, y0, D, Lo, C, f, stream=None):
    """Device tensors in, device tensors out (see include/pf.h)."""
    rc = load().pf_ivp_trapezoid_system(m, steps, _ptr(L), float(h), _ptr(g), _ptr(y0), _ptr(D),
                                        _ptr(Lo), _ptr(C), _ptr(f), _stream(stream))
    if rc != 0:
        raise PFError(rc, "pf_ivp_trapezoid_system")


def pf_ivp_solve(m, L, t0, T, p, N, g, y0, y, opts=None, stream=None):
    """Time-parallel trapezoid solution of y' = L y + g(t) on a coarse mesh of
    p sub-intervals of N steps; returns pf_info.  L (m*m, column-major), g
    ((p*N+1)*m), y0 (m) and y ((p*N+1)*m) are device tensors."""
    info = pf_info()
    rc = load().pf_ivp_solve(m, _ptr(L), float(t0), float(T), p, N, _ptr(g), _ptr(y0), _ptr(y),
                             ctypes.byref(opts) if opts is not None else None, _stream(stream),
                             ctypes.byref(info))
    if rc < 0 or rc in (PF_ENOMEM, PF_EHIP, PF_EUNSUPPORTED):
        raise PFError(rc, "pf_ivp_solve")
    return info


def pf_ivp_create(m, p, N, opts=None, stream=None):
    """A plan (opaque handle) for IVPs of this shape; free with pf_ivp_destroy."""
    h = ctypes.c_void_p()
    rc = load().pf_ivp_create(m, p, N, ctypes.byref(opts) if opts is not None else None,
                              _stream(stream), ctypes.byref(h))
    if rc != 0:
        raise PFError(rc, "pf_ivp_create")
    return h


def pf_ivp_run(plan, L, t0, T, g, y0, y, stream=None, want_info=True):
    """Solve with a plan; returns pf_info (synchronizing) or None."""
    info = pf_info() if want_info else None
    rc = load().pf_ivp_run(plan, _ptr(L), float(t0), float(T), _ptr(g), _ptr(y0), _ptr(y),
                           _stream(stream), ctypes.byref(info) if info is not None else None)
    if rc < 0 or rc in (PF_ENOMEM, PF_EHIP, PF_EUNSUPPORTED):
        raise PFError(rc, "pf_ivp_run")
    return info


def pf_ivp_destroy(plan):
    load().pf_ivp_destroy(plan)


def pf_solve_batch(mats, opts, nrhs, fs, xs, stream=None, keep_factors=False, factors=None):
    """mats: list of pf_matrix; fs/xs: lists of device tensors (nrhs_i, n_i).
    factors: optional list of existing handles (or None) per system: those
    systems are solved with their handle instead of being factored.  With
    keep_factors (or factors) the returned list holds every system's handle
    (the existing ones as given, the new ones for the caller to destroy)."""
    lib = load()
    ns = len(mats)
    A, nr, fp, lf, xp, lx = _batch_arrays(mats, nrhs, fs, xs)
    fac = None
    if keep_factors or factors is not None:
        fac = (ctypes.c_void_p * ns)()
        if factors is not None:
            for i, h in enumerate(factors):
                fac[i] = None if h is None else (h.value if isinstance(h, ctypes.c_void_p) else h)
    infos = (pf_info * ns)()
    rc = lib.pf_solve_batch(ns, A, ctypes.byref(opts) if opts is not None else None, nr, fp, lf,
                            xp, lx, _stream(stream), fac, infos)
    if rc < 0 or rc in (PF_ENOMEM, PF_EHIP, PF_EUNSUPPORTED):
        raise PFError(rc, "pf_solve_batch")
    out = None
    if fac is not None:
        out = [None if v is None else ctypes.c_void_p(v) for v in fac]
    return list(infos), out


def _batch_arrays(mats, nrhs, fs, xs):
    ns = len(mats)
    A = (pf_matrix * ns)(*mats)
    nr = (ctypes.c_int32 * ns)(*nrhs)
    fp = (ctypes.c_void_p * ns)(*[f.data_ptr() for f in fs])
    xp = (ctypes.c_void_p * ns)(*[x.data_ptr() for x in xs])
    lf = (ctypes.c_int64 * ns)(*[f.shape[-1] for f in fs])
    lx = (ctypes.c_int64 * ns)(*[x.shape[-1] for x in xs])
    return A, nr, fp, lf, xp, lx


class Batch:
    """pf_batch_create / pf_batch_run / pf_batch_factor / pf_batch_destroy.

    mats: list of pf_matrix; fs/xs: device tensors (nrhs_i, n_i) per system
    (the batch keeps their pointers: keep the tensors alive)."""

    def __init__(self, mats, opts, nrhs, fs, xs, stream=None):
        lib = load()
        self.n = len(mats)
        self._keep = (mats, fs, xs)
        self._arrays = _batch_arrays(mats, nrhs, fs, xs)
        h = ctypes.c_void_p()
        rc = lib.pf_batch_create(self.n, *self._arrays[:1],
                                 ctypes.byref(opts) if opts is not None else None,
                                 *self._arrays[1:], _stream(stream), ctypes.byref(h))
        if rc != 0:
            raise PFError(rc, "pf_batch_create")
        self.h = h

    def run(self, stream=None, want_info=True):
        infos = (pf_info * self.n)() if want_info else None
        rc = load().pf_batch_run(self.h, _stream(stream), infos)
        if rc < 0 or rc in (PF_ENOMEM, PF_EHIP, PF_EUNSUPPORTED):
            raise PFError(rc, "pf_batch_run")
        return list(infos) if want_info else None

    def profile(self, stream=None):
        """Per grouped launch: dicts of pf_launch_info (phase, level, kind, m,
        f32, mapping, rows, rhs_rows, workgroups, ms)."""
        n = 4096
        buf = (pf_launch_info * n)()
        cnt = ctypes.c_int32()
        rc = load().pf_batch_profile(self.h, _stream(stream), n, buf, ctypes.byref(cnt))
        if rc != 0:
            raise PFError(rc, "pf_batch_profile")
        return [buf[i].as_dict() for i in range(min(cnt.value, n))]

    def factor(self, i):
        out = ctypes.c_void_p()
        rc = load().pf_batch_factor(self.h, i, ctypes.byref(out))
        if rc != 0:
            raise PFError(rc, "pf_batch_factor")
        return out

    def destroy(self):
        if self.h:
            load().pf_batch_destroy(self.h)
            self.h = None


def pf_autotune(A: pf_matrix, base: pf_opts | None = None, nrhs: int = 1, stream=None):
    """Fastest launch shape for A (pf_opts, median ms of pf_factor_solve)."""
    best = pf_opts()
    ms = ctypes.c_float()
    rc = load().pf_autotune(ctypes.byref(A), ctypes.byref(base) if base is not None else None,
                            nrhs, _stream(stream), ctypes.byref(best), ctypes.byref(ms))
    if rc != 0:
        raise PFError(rc, "pf_autotune")
    return best, float(ms.value)


def pf_autotune_clear():
    load().pf_autotune_clear()


class pf_request(ctypes.Structure):
    _fields_ = [("A", pf_matrix), ("nrhs", ctypes.c_int32), ("keep", ctypes.c_int32),
                ("f", ctypes.c_void_p), ("ldf", ctypes.c_int64), ("x", ctypes.c_void_p),
                ("ldx", ctypes.c_int64), ("factor", ctypes.c_int64), ("after", ctypes.c_void_p)]


class pf_server_info(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_size_t), ("used", ctypes.c_size_t), ("queued", ctypes.c_int64),
                ("inflight", ctypes.c_int64), ("resident", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("setup_ms_max", ctypes.c_double), ("setup_ms_total", ctypes.c_double),
                ("launch_ms_max", ctypes.c_double), ("launch_ms_total", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _server_sigs(lib):
    vp, i32, i64, P = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER
    d = ctypes.c_double
    sigs = {
        "pf_server_create": (ctypes.c_int, [ctypes.c_size_t, P(pf_opts), i32, i32, P(vp)]),
        "pf_server_submit": (ctypes.c_int, [vp, P(pf_request), P(i64)]),
        "pf_server_poll": (ctypes.c_int, [vp, i64, P(pf_info)]),
        "pf_server_wait": (ctypes.c_int, [vp, i64, P(pf_info)]),
        "pf_server_times": (ctypes.c_int, [vp, i64, P(d), P(d), P(d)]),
        "pf_server_release": (ctypes.c_int, [vp, i64]),
        "pf_server_reserve": (ctypes.c_int, [vp, ctypes.c_size_t]),
        "pf_server_stats": (ctypes.c_int, [vp, P(pf_server_info)]),
        "pf_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args


class Server:
    """pf_server_*: continuous batching of factor-and-solve requests under a
    device-memory budget, with resident factors for repeat right-hand sides."""

    def __init__(self, budget_bytes, opts=None, max_inflight=0, nstreams=0):
        lib = load()
        _server_sigs(lib)
        h = ctypes.c_void_p()
        rc = lib.pf_server_create(budget_bytes, ctypes.byref(opts) if opts is not None else None,
                                  max_inflight, nstreams, ctypes.byref(h))
        if rc != 0:
            raise PFError(rc, "pf_server_create")
        self.h = h
        self._keep = {}

    def submit(self, A, f, x, keep=False, factor=-1, stream=None):
        """A: pf_matrix; f, x: device tensors (nrhs, n).  The request runs
        after the work queued so far on `stream` (torch's current stream by
        default), which is where A and f were produced."""
        nrhs = 1 if f.dim() == 1 else f.shape[0]
        req = pf_request(A, nrhs, 1 if keep else 0, f.data_ptr(), f.shape[-1], x.data_ptr(),
                         x.shape[-1], factor, _stream(stream))
        t = ctypes.c_int64()
        rc = load().pf_server_submit(self.h, ctypes.byref(req), ctypes.byref(t))
        if rc != 0:
            raise PFError(rc, "pf_server_submit")
        self._keep[t.value] = (f, x)
        return t.value

    def poll(self, ticket):
        info = pf_info()
        rc = load().pf_server_poll(self.h, ticket, ctypes.byref(info))
        if rc < 0:
            raise PFError(rc, "pf_server_poll")
        return info if rc == 1 else None

    def wait(self, ticket):
        info = pf_info()
        rc = load().pf_server_wait(self.h, ticket, ctypes.byref(info))
        if rc < 0 or rc in (PF_EHIP,):
            raise PFError(rc, "pf_server_wait")
        return info

    def times(self, ticket):
        s, a, d = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        load().pf_server_times(self.h, ticket, ctypes.byref(s), ctypes.byref(a), ctypes.byref(d))
        return s.value, a.value, d.value

    def reserve(self, nbytes):
        rc = load().pf_server_reserve(self.h, int(nbytes))
        if rc != 0:
            raise PFError(rc, "pf_server_reserve")

    def release(self, factor):
        rc = load().pf_server_release(self.h, factor)
        if rc != 0:
            raise PFError(rc, "pf_server_release")

    def stats(self):
        st = pf_server_info()
        load().pf_server_stats(self.h, ctypes.byref(st))
        return st.as_dict()

    def destroy(self):
        if self.h:
            load().pf_server_destroy(self.h)
            self.h = None
