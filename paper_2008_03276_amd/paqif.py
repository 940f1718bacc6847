"""Torch-facing wrappers of the PAQIF entry points (marshalling only).

Inputs are CUDA (HIP) tensors; the library works on the current torch
stream and never allocates: workspaces are allocated here with torch and
passed in.  Band layout: ``band[i, d] = a(i, i+d-q)`` for the concatenated
rows of all systems, ``offsets`` the int64 row offsets (count+1 entries).
"""
import ctypes

import torch

from . import _binding as B

_HANDLES = {}


def handle(device=None):
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    h = _HANDLES.get(dev)
    if h is None:
        with torch.cuda.device(dev):
            hv = ctypes.c_void_p()
            B.check(B.lib().paqif_create(ctypes.byref(hv)), "paqif_create")
        h = hv.value
        _HANDLES[dev] = h
    return h


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")


def _need_len(t, n, name):
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, the batch needs {n}")


def _check_system_args(batch, band, b=None, bounded=None):
    """Sizes of the per-row arguments against the batch (the C ABI takes
    bare pointers, so a short buffer would be read or written past its end)."""
    rows = batch.total_rows
    _need(band, torch.float64, "band")
    _need_len(band, rows * (2 * batch.q + 1), "band")
    if b is not None:
        _need(b, torch.float64, "b")
        _need_len(b, rows, "b")
    if bounded is not None:
        _need(bounded, torch.uint8, "bounded")
        _need_len(bounded, rows, "bounded")


def _check_workspace(batch, workspace, prec, mode):
    if not (workspace.is_cuda and workspace.is_contiguous()):
        raise ValueError("workspace must be a contiguous CUDA tensor")
    have = workspace.numel() * workspace.element_size()
    need = batch.workspace_bytes(prec, mode)
    if have < need:
        raise ValueError(f"workspace has {have} bytes, the batch needs {need}")


class Batch:
    """Host + device description of a batch of band systems (one q)."""

    def __init__(self, offsets, q, device=None, order=None):
        offs = torch.as_tensor(offsets, dtype=torch.int64).cpu()
        self.count = int(offs.numel() - 1)
        self.q = int(q)
        sizes = offs[1:] - offs[:-1]
        self.max_n = int(sizes.max()) if self.count > 0 else 0
        self.total_rows = int(offs[-1]) if self.count > 0 else 0
        device = device or torch.device("cuda", torch.cuda.current_device())
        self.offsets = offs.to(device)
        if order == "lpt":  # largest systems first
            order = torch.argsort(sizes, descending=True, stable=True).to(torch.int32)
        self.order = None if order is None else torch.as_tensor(order, dtype=torch.int32).to(device)
        self.sizes = sizes
        self.c = B.PaqifBatch(self.count, self.q, self.offsets.data_ptr(), self.max_n,
                              self.total_rows,
                              self.order.data_ptr() if self.order is not None else None)

    def workspace_bytes(self, prec=B.PREC_FP64, mode=B.LCP_EXACT):
        n = B.lib().paqif_workspace_bytes(handle(), ctypes.byref(self.c), prec, mode)
        if n == 0 and self.count > 0:
            raise ValueError("invalid batch description")
        return int(n)

    def workspace(self, prec=B.PREC_FP64, mode=B.LCP_EXACT):
        return torch.empty(self.workspace_bytes(prec, mode), dtype=torch.uint8,
                           device=self.offsets.device)


def solve_lcp(batch, band, b, mode=B.LCP_EXACT, prec=B.PREC_FP64, bounded=None,
              refine_tol=1e-10, max_iter=64, workspace=None, want_w=True, want_active=True,
              u=None):
    """PAQIF solve of the banded LCP for every system of ``batch``.

    With mode=LCP_EXACT_FROM_U, ``u`` (the iterate of ``start_sweeps``) is
    the start and is overwritten by the solution.
    Returns dict(u, w, active, status, iters) (device tensors)."""
    _check_system_args(batch, band, b, bounded)
    dev = band.device
    n = batch.total_rows
    if mode == B.LCP_EXACT_FROM_U:
        if u is None:
            raise ValueError("mode LCP_EXACT_FROM_U needs the start iterate u")
        _need(u, torch.float64, "u")
        _need_len(u, n, "u")
    elif u is not None:
        raise ValueError("u is an input only with mode LCP_EXACT_FROM_U")
    else:
        u = torch.empty(n, dtype=torch.float64, device=dev)
    w = torch.empty(n, dtype=torch.float64, device=dev) if want_w else None
    act = torch.empty(n, dtype=torch.uint8, device=dev) if want_active else None
    st = torch.empty(batch.count, dtype=torch.int32, device=dev)
    it = torch.empty(batch.count, dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = batch.workspace(prec, mode)
    _check_workspace(batch, workspace, prec, mode)
    code = B.lib().paqif_solve_lcp(handle(), ctypes.byref(batch.c), _ptr(band), _ptr(b),
                                   _ptr(bounded), mode, prec, refine_tol, max_iter, _ptr(u),
                                   _ptr(w), _ptr(act), _ptr(st), _ptr(it), _ptr(workspace),
                                   _stream())
    B.check(code, "paqif_solve_lcp")
    return dict(u=u, w=w, active=act, status=st, iters=it)


def solve_lcp_noalloc(batch, band, b, u, status, mode=B.LCP_EXACT, prec=B.PREC_FP64,
                      bounded=None, refine_tol=1e-10, max_iter=64, w=None, active=None,
                      iters=None):
    """The allocation-free entry point: same solve as ``solve_lcp``, its
    scratch in the library's own device array; the caller passes every
    output (``u``, ``status`` and optionally ``w``, ``active``, ``iters``),
    so nothing is allocated here either.  Returns the call status code
    (PAQIF_EWORKSPACE when the batch exceeds the library's scratch)."""
    _check_system_args(batch, band, b, bounded)
    rows = batch.total_rows
    _need(u, torch.float64, "u")
    _need_len(u, rows, "u")
    _need(status, torch.int32, "status")
    _need_len(status, batch.count, "status")
    if w is not None:
        _need(w, torch.float64, "w")
        _need_len(w, rows, "w")
    if active is not None:
        _need(active, torch.uint8, "active")
        _need_len(active, rows, "active")
    if iters is not None:
        _need(iters, torch.int32, "iters")
        _need_len(iters, batch.count, "iters")
    return B.lib().paqif_solve_lcp_noalloc(handle(), ctypes.byref(batch.c), _ptr(band), _ptr(b),
                                           _ptr(bounded), mode, prec, refine_tol, max_iter,
                                           _ptr(u), _ptr(w), _ptr(active), _ptr(status),
                                           _ptr(iters), _stream())


def solve_lcp_many(calls, mode=B.LCP_EXACT, prec=B.PREC_FP64, refine_tol=1e-10, max_iter=64,
                   want_w=True, want_active=True):
    """Several ``solve_lcp`` calls in one (paqif_solve_lcp_many): ``calls`` is
    a list of dicts with keys batch, band, b and optionally bounded,
    workspace (distinct per call) and u (the start with LCP_EXACT_FROM_U).
    Every call's start sweeps run first, then the FP64 row-layout solves of
    all calls in one launch.  Returns one result dict per call, as
    ``solve_lcp``."""
    if len(calls) > B.MAX_LCP_CALLS:
        raise ValueError(f"at most {B.MAX_LCP_CALLS} calls")
    arr = (B.PaqifLcpCall * max(len(calls), 1))()
    out = []
    keep = []
    for i, c in enumerate(calls):
        batch, band, b = c["batch"], c["band"], c["b"]
        bounded = c.get("bounded")
        _check_system_args(batch, band, b, bounded)
        dev = band.device
        n = batch.total_rows
        u = c.get("u")
        if mode == B.LCP_EXACT_FROM_U:
            if u is None:
                raise ValueError("mode LCP_EXACT_FROM_U needs the start iterate u")
            _need(u, torch.float64, "u")
            _need_len(u, n, "u")
        elif u is not None:
            raise ValueError("u is an input only with mode LCP_EXACT_FROM_U")
        else:
            u = torch.empty(n, dtype=torch.float64, device=dev)
        w = torch.empty(n, dtype=torch.float64, device=dev) if want_w else None
        act = torch.empty(n, dtype=torch.uint8, device=dev) if want_active else None
        st = torch.empty(batch.count, dtype=torch.int32, device=dev)
        it = torch.empty(batch.count, dtype=torch.int32, device=dev)
        ws = c.get("workspace")
        if ws is None:
            ws = batch.workspace(prec, mode)
        _check_workspace(batch, ws, prec, mode)
        arr[i] = B.PaqifLcpCall(ctypes.pointer(batch.c), _ptr(band), _ptr(b), _ptr(bounded),
                                _ptr(u), _ptr(w), _ptr(act), _ptr(st), _ptr(it), _ptr(ws))
        keep.append(ws)
        out.append(dict(u=u, w=w, active=act, status=st, iters=it))
    code = B.lib().paqif_solve_lcp_many(handle(), len(calls), arr, mode, prec, refine_tol,
                                        max_iter, _stream())
    B.check(code, "paqif_solve_lcp_many")
    return out


def start_sweeps(batch, band, b, prec=B.PREC_FP64, bounded=None, workspace=None, u=None):
    """The exact LCP's starting iterate alone (the handle's start sweeps for
    (q, prec)); pass it to ``solve_lcp(..., mode=LCP_EXACT_FROM_U, u=u)``.
    ``workspace``: as for solve_lcp in mode LCP_EXACT (its record area holds
    the iterate between launches).  Returns u."""
    _check_system_args(batch, band, b, bounded)
    if u is None:
        u = torch.empty(batch.total_rows, dtype=torch.float64, device=band.device)
    _need(u, torch.float64, "u")
    _need_len(u, batch.total_rows, "u")
    if workspace is None:
        workspace = batch.workspace(prec, B.LCP_EXACT)
    _check_workspace(batch, workspace, prec, B.LCP_EXACT)
    code = B.lib().paqif_start_sweeps(handle(), ctypes.byref(batch.c), _ptr(band), _ptr(b),
                                      _ptr(bounded), int(prec), _ptr(u), _ptr(workspace),
                                      _stream())
    B.check(code, "paqif_start_sweeps")
    return u


def factor(batch, band, pinned=None, factors=None, prec=B.PREC_FP64):
    """A = W0 Z0 for every system (records in FP64, or FP32 for
    prec=PREC_FP32_IR); returns (factors, status)."""
    _check_system_args(batch, band, bounded=pinned)
    if factors is None:
        factors = batch.workspace(prec, B.LCP_LINEAR)
    _check_workspace(batch, factors, prec, B.LCP_LINEAR)
    st = torch.empty(batch.count, dtype=torch.int32, device=band.device)
    code = B.lib().paqif_factor(handle(), ctypes.byref(batch.c), _ptr(band), _ptr(pinned),
                                int(prec), _ptr(factors), _ptr(st), _stream())
    B.check(code, "paqif_factor")
    return factors, st


def solve_factored(batch, factors, rhs, pinned=None, prec=B.PREC_FP64):
    """x = (W0 Z0)^{-1} rhs with the records of factor(..., prec=prec)."""
    _need(rhs, torch.float64, "rhs")
    _need_len(rhs, batch.total_rows, "rhs")
    if pinned is not None:
        _need(pinned, torch.uint8, "pinned")
        _need_len(pinned, batch.total_rows, "pinned")
    _check_workspace(batch, factors, prec, B.LCP_LINEAR)
    x = torch.empty_like(rhs)
    code = B.lib().paqif_solve_factored(handle(), ctypes.byref(batch.c), _ptr(factors), int(prec),
                                        _ptr(pinned), _ptr(rhs), _ptr(x), _stream())
    B.check(code, "paqif_solve_factored")
    return x


def layout_count(q):
    return B.lib().paqif_layout_count(int(q))


def set_layout(q, prec, layout):
    B.check(B.lib().paqif_set_layout(handle(), int(q), int(prec), int(layout)), "paqif_set_layout")


def get_layout(q, prec=B.PREC_FP64):
    return B.lib().paqif_get_layout(handle(), int(q), int(prec))


def set_start_sweeps(q, prec, sweeps):
    """Projected Jacobi sweeps that choose the exact LCP's starting active
    set for (q, prec) on this process's handle (0: the sign of b)."""
    B.check(B.lib().paqif_set_start_sweeps(handle(), int(q), int(prec), int(sweeps)),
            "paqif_set_start_sweeps")


def get_start_sweeps(q, prec=B.PREC_FP64):
    return B.lib().paqif_get_start_sweeps(handle(), int(q), int(prec))


def autotune(batch, band, b, mode=B.LCP_EXACT, prec=B.PREC_FP64, bounded=None, max_iter=64,
             workspace=None):
    """Time every lane layout of the LCP kernel on this batch; the fastest is
    kept in the handle for (q, prec); in exact mode the start sweeps are then
    tuned with that layout (get_start_sweeps).  Returns (chosen layout,
    times_ms per layout)."""
    _check_system_args(batch, band, b, bounded)
    nl = layout_count(batch.q)
    times = (ctypes.c_float * nl)()
    u = torch.empty(batch.total_rows, dtype=torch.float64, device=band.device)
    st = torch.empty(batch.count, dtype=torch.int32, device=band.device)
    if workspace is None:
        workspace = batch.workspace(prec, mode)
    _check_workspace(batch, workspace, prec, mode)
    B.check(B.lib().paqif_autotune(handle(), ctypes.byref(batch.c), _ptr(band), _ptr(b),
                                   _ptr(bounded), mode, prec, max_iter, _ptr(u), _ptr(st),
                                   _ptr(workspace), _stream(), times), "paqif_autotune")
    return get_layout(batch.q, prec), [float(t) for t in times]


def partitioned_workspace_bytes(n, q, r):
    return int(B.lib().paqif_partitioned_workspace_bytes(int(n), int(q), int(r)))


def solve_partitioned(band, b, r, mode=B.LCP_LINEAR, bounded=None, max_iter=64, workspace=None):
    """Partitioned PAQIF solve of one long band system over r blocks
    (``band``: (n, 2q+1) FP64 device tensor, ``b``: (n,)).  Returns
    dict(u, active, status, iters) with status and iters one-element int32
    device tensors.  The exact mode synchronises the current stream."""
    _need(band, torch.float64, "band")
    _need(b, torch.float64, "b")
    if bounded is not None:
        _need(bounded, torch.uint8, "bounded")
    n, w = int(band.shape[0]), int(band.shape[1])
    q = (w - 1) // 2
    if tuple(b.shape) != (n,) or w != 2 * q + 1:
        raise ValueError("band must be (n, 2q+1) and b (n,)")
    dev = band.device
    u = torch.empty(n, dtype=torch.float64, device=dev)
    act = torch.empty(n, dtype=torch.uint8, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    it = torch.empty(1, dtype=torch.int32, device=dev)
    if workspace is None:
        nb = partitioned_workspace_bytes(n, q, r)
        workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    code = B.lib().paqif_solve_partitioned(handle(), n, q, int(r), _ptr(band), _ptr(b),
                                           _ptr(bounded), int(mode), int(max_iter), _ptr(u),
                                           _ptr(act), _ptr(st), _ptr(it), _ptr(workspace),
                                           _stream())
    B.check(code, "paqif_solve_partitioned")
    return dict(u=u, active=act, status=st, iters=it)
