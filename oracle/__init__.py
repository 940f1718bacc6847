"""Oracle: plain, slow, FP64 CPU reference of the PAQIF / EHL hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product library
(``paper_2008_03276_amd``) never imports, links or calls anything here, and
this package never imports the product.

Parts:
  * ``aqif_lcp.c`` (ctypes below): banded AQIF factor/solve and the banded
    LCP (Sec. 2.1-2.2 of the paper; projected splitting of Sec. 3.2).
  * ``deform.py``: elastic deformation kernels and sums (Sec. 3.3.1).
  * ``ehl_line.py`` / ``ehl_point.py``: EHL residual, band Jacobian,
    hybrid Newton line iteration and load balance (Sec. 3.3).
  * ``partitioned.py``: the partitioned PAQIF solve of one long band
    system (Sec. 2.1-2.2, Steps 1-7).
  * ``convdiff.py``: the linear convection-diffusion workload of the
    numerical results (kappa-schemes, line relaxation with banded solves).
"""
import ctypes
import os

import numpy as np

from . import build as _build

OK, ZERO_PIVOT, NONFINITE, LCP_NOT_CONVERGED = 0, 1, 2, 3
LINEAR, CLIP, EXACT = 0, 1, 2

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = ctypes.CDLL(path)
        d, i64, i32, u8 = (ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int,
                           ctypes.POINTER(ctypes.c_uint8))
        L.or_aqif_solve.argtypes = [i64, i32, d, u8, d, d]
        L.or_aqif_factor_dense.argtypes = [i64, i32, d, u8, d, d]
        L.or_lcp_solve.argtypes = [i64, i32, d, d, u8, i32, i32, d, d, u8,
                                   ctypes.POINTER(ctypes.c_int)]
        L.or_lcp_solve_start.argtypes = [i64, i32, d, d, u8, u8, i32, d, d, u8,
                                         ctypes.POINTER(ctypes.c_int)]
        L.or_lcp_pgs.argtypes = [i64, i32, d, d, u8, ctypes.c_double, i32, ctypes.c_double, d,
                                 ctypes.POINTER(ctypes.c_int)]
        L.or_start_sweeps.argtypes = [i64, i32, d, d, u8, i32, d]
        L.or_lcp_batch.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_int64), d, d, u8, i32, i32,
                                   d, d, u8, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), i32]
        for f in (L.or_aqif_solve, L.or_aqif_factor_dense, L.or_lcp_solve, L.or_lcp_solve_start,
                  L.or_lcp_pgs, L.or_lcp_batch, L.or_start_sweeps):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_uint8)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _mask(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def aqif_solve(band, f, pinned=None):
    """x = A_eff^{-1} f_eff by the centre-out AQIF elimination (Sec. 2.2).

    ``band``: (n, 2q+1) with band[i, d] = a(i, i+d-q).  Rows/columns marked
    in ``pinned`` are replaced by the identity and f_i by 0.
    Returns (x, status)."""
    band = _f64(band)
    n, w = band.shape
    q = (w - 1) // 2
    f = _f64(f)
    pinned = _mask(pinned)
    x = np.zeros(n)
    st = lib().or_aqif_solve(n, q, _dp(band), _u8(pinned), _dp(f), _dp(x))
    return x, st


def aqif_factor_dense(band, pinned=None):
    """Dense W0 (unit 'hourglass') and Z0 ('butterfly') with A = W0 Z0."""
    band = _f64(band)
    n, w = band.shape
    q = (w - 1) // 2
    pinned = _mask(pinned)
    W = np.zeros((n, n))
    Z = np.zeros((n, n))
    st = lib().or_aqif_factor_dense(n, q, _dp(band), _u8(pinned), _dp(W), _dp(Z))
    return W, Z, st


def lcp_solve(band, f, bounded=None, mode=EXACT, max_iter=64):
    """Banded LCP u >= 0, w = A u - f >= 0, u.w = 0 (Sec. 2.1 eq. 14).

    Returns dict(u, w, active, iters, status)."""
    band = _f64(band)
    n, wd = band.shape
    q = (wd - 1) // 2
    f = _f64(f)
    bounded = _mask(bounded)
    u = np.zeros(n)
    w = np.zeros(n)
    act = np.zeros(n, dtype=np.uint8)
    it = ctypes.c_int(0)
    st = lib().or_lcp_solve(n, q, _dp(band), _dp(f), _u8(bounded), mode, max_iter, _dp(u),
                            _dp(w), _u8(act), ctypes.byref(it))
    return dict(u=u, w=w, active=act, iters=it.value, status=st)


def lcp_solve_start(band, f, bounded=None, start=None, max_iter=64):
    """Exact banded LCP by the active-set iteration from the start set
    ``start`` (None: the empty set).  Returns dict(u, w, active, iters,
    status)."""
    band = _f64(band)
    n, wd = band.shape
    q = (wd - 1) // 2
    f = _f64(f)
    bounded = _mask(bounded)
    start = _mask(start)
    u = np.zeros(n)
    w = np.zeros(n)
    act = np.zeros(n, dtype=np.uint8)
    it = ctypes.c_int(0)
    st = lib().or_lcp_solve_start(n, q, _dp(band), _dp(f), _u8(bounded), _u8(start), max_iter,
                                  _dp(u), _dp(w), _u8(act), ctypes.byref(it))
    return dict(u=u, w=w, active=act, iters=it.value, status=st)


def start_sweeps(band, f, bounded=None, k=1):
    """Iterate after k projected Jacobi sweeps from u = 0 (the exact LCP's
    start rule: A_0 = {bounded i : u_i <= 0}); not part of the paper's
    method."""
    band = _f64(band)
    n, wd = band.shape
    q = (wd - 1) // 2
    f = _f64(f)
    bounded = _mask(bounded)
    u = np.zeros(n)
    lib().or_start_sweeps(n, q, _dp(band), _dp(f), _u8(bounded), int(k), _dp(u))
    return u


def lcp_start_sets(q, offsets, band, f, bounded=None, k=0, frac=0.0):
    """Per-system starting active sets of a batch: the systems with at
    least int(frac * (max_n // 2)) elimination levels (n // 2; frac = 0:
    every system) from k start sweeps, the others (and all for k == 0) from
    the sign of f."""
    offsets = np.asarray(offsets, dtype=np.int64)
    band = _f64(band).reshape(-1, 2 * q + 1)
    f = _f64(f)
    bnd = np.ones(len(f), dtype=bool) if bounded is None else np.asarray(bounded) != 0
    sizes = np.diff(offsets)
    lmin = int(frac * float(int(sizes.max()) // 2)) if len(sizes) else 0
    start = np.zeros(len(f), dtype=np.uint8)
    for s in range(len(sizes)):
        a, b = int(offsets[s]), int(offsets[s + 1])
        if k > 0 and (b - a) // 2 >= lmin:
            u = start_sweeps(band[a:b], f[a:b], None if bounded is None else bounded[a:b], k)
            start[a:b] = bnd[a:b] & (u <= 0.0)
        else:
            start[a:b] = bnd[a:b] & (f[a:b] <= 0.0)
    return start


def lcp_pgs(band, f, bounded=None, omega=1.0, max_sweeps=100000, tol=1e-14):
    """Projected SOR (Cryer) for the same LCP; independent of AQIF."""
    band = _f64(band)
    n, wd = band.shape
    q = (wd - 1) // 2
    f = _f64(f)
    bounded = _mask(bounded)
    u = np.zeros(n)
    sw = ctypes.c_int(0)
    st = lib().or_lcp_pgs(n, q, _dp(band), _dp(f), _u8(bounded), omega, max_sweeps, tol,
                          _dp(u), ctypes.byref(sw))
    return u, st, sw.value


def lcp_batch(q, offsets, band, f, bounded=None, mode=EXACT, max_iter=64, nthreads=None):
    """Batch of band LCPs (systems concatenated by ``offsets``)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    count = len(offsets) - 1
    total = int(offsets[-1])
    band = _f64(band).reshape(total, 2 * q + 1)
    f = _f64(f)
    bounded = _mask(bounded)
    u = np.zeros(total)
    w = np.zeros(total)
    act = np.zeros(total, dtype=np.uint8)
    status = np.zeros(count, dtype=np.int32)
    iters = np.zeros(count, dtype=np.int32)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    lib().or_lcp_batch(count, q, offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                       _dp(band), _dp(f), _u8(bounded), mode, max_iter, _dp(u), _dp(w),
                       _u8(act), status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                       iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nthreads)
    return dict(u=u, w=w, active=act, status=status, iters=iters)
