"""Torch-facing wrappers of the EHL entry points (marshalling only).

Pressure fields of B line-contact instances on one grid are (B, N) tensors
(row b = instance b), which is the column-major N x B layout of the C ABI.
"""
import ctypes
import math

import torch

from . import _binding as B
from .paqif import _need, _ptr, _stream, handle

XA, XB = -4.5, 1.5


def line_grid(N, x0=XA, x1=XB):
    return B.EhlGrid(int(N), 1, float(x0), float(x1), 0.0, 0.0)


def point_grid(Nx, Ny, x0=XA, x1=XB, y0=-3.0, y1=3.0):
    return B.EhlGrid(int(Nx), int(Ny), float(x0), float(x1), float(y0), float(y1))


def default_opts(**kw):
    o = dict(omega=0.5, c_h0=0.1, switch_ratio=0.6, tol=1e-13, max_newton=4000, kernel_terms=2,
             lcp_max_iter=64, deform_prec=B.PREC_FP64, lcp_prec=B.PREC_FP64, steps_per_graph=16,
             start_rule=1, limiter_jacobian=2, stall_steps=0, convection=0, kappa=0.0,
             lcp_fail_steps=16, splitting=0)
    o.update(kw)
    return B.EhlOpts(**o)


def params_tensor(M, L, device):
    M = torch.as_tensor(M, dtype=torch.float64).reshape(-1)
    L = torch.as_tensor(L, dtype=torch.float64).reshape(-1)
    return torch.stack([M, L], dim=1).contiguous().to(device)


def deformation(P, grid, prec=B.PREC_FP64):
    """H_el of the pressure fields P: (B, N) for a line grid, (B, Nx, Ny)
    for a point grid."""
    _need(P, torch.float64, "P")
    nb = P.shape[0]
    out = torch.empty_like(P)
    ws = torch.empty(max(1, B.lib().ehl_deformation_workspace_bytes(ctypes.byref(grid), nb)),
                     dtype=torch.uint8, device=P.device)
    B.check(B.lib().ehl_deformation(handle(), ctypes.byref(grid), _ptr(P), nb, prec, _ptr(out),
                                    _ptr(ws), _stream()), "ehl_deformation")
    return out


def assemble(grid, params, P, Hel, H0, opts=None, rough=None):
    """Residual, band (-dR/dsigma), rhs, bounded and direct masks."""
    opts = opts or default_opts()
    for t, name in ((P, "P"), (Hel, "Hel"), (H0, "H0"), (params, "params")):
        _need(t, torch.float64, name)
    if rough is not None:
        _need(rough, torch.float64, "rough")
    nb, N = P.shape
    n = N - 2
    dev = P.device
    R = torch.empty(nb, n, dtype=torch.float64, device=dev)
    band = torch.empty(nb, n, 9, dtype=torch.float64, device=dev)
    rhs = torch.empty(nb, n, dtype=torch.float64, device=dev)
    bounded = torch.empty(nb, n, dtype=torch.uint8, device=dev)
    direct = torch.empty(nb, N, dtype=torch.uint8, device=dev)
    B.check(B.lib().ehl_jacobian_assemble(handle(), ctypes.byref(grid), _ptr(params), nb,
                                          ctypes.byref(opts), _ptr(P), _ptr(Hel), _ptr(H0),
                                          _ptr(rough), _ptr(R), _ptr(band), _ptr(rhs),
                                          _ptr(bounded), _ptr(direct), _stream()),
            "ehl_jacobian_assemble")
    return dict(R=R, band=band, rhs=rhs, bounded=bounded, direct=direct)


def solve_line(M, L, N, opts=None, rough=None, P=None, H0=None, device=None, stream=None):
    """Hybrid Newton line iteration for B = len(M) instances on one grid.

    Runs on a private stream (so the steps can be captured in HIP graphs).
    Returns dict(P, H0, H, Hmin, status, iters) as device tensors."""
    opts = opts or default_opts()
    device = device or torch.device("cuda", torch.cuda.current_device())
    grid = line_grid(N)
    params = params_tensor(M, L, device)
    nb = params.shape[0]
    if P is None:
        P = torch.zeros(nb, N, dtype=torch.float64, device=device)
    else:
        P = P.clone().contiguous()
    H0 = torch.zeros(nb, dtype=torch.float64, device=device) if H0 is None else \
        torch.as_tensor(H0, dtype=torch.float64, device=device).clone()
    H = torch.empty(nb, N, dtype=torch.float64, device=device)
    Hmin = torch.empty(nb, dtype=torch.float64, device=device)
    status = torch.empty(nb, dtype=torch.int32, device=device)
    iters = torch.empty(nb, dtype=torch.int32, device=device)
    nbytes = B.lib().ehl_newton_workspace_bytes(handle(), ctypes.byref(grid), nb,
                                                ctypes.byref(opts))
    if nbytes == 0:
        raise ValueError("invalid EHL grid/options")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    if rough is not None:
        _need(rough, torch.float64, "rough")
    s = stream or torch.cuda.Stream(device=device)
    s.wait_stream(torch.cuda.current_stream(device))
    with torch.cuda.stream(s):
        code = B.lib().ehl_newton_tvd(handle(), ctypes.byref(grid), _ptr(params), nb,
                                      ctypes.byref(opts), _ptr(rough), _ptr(P), _ptr(H0),
                                      _ptr(H), _ptr(Hmin), _ptr(status), _ptr(iters), _ptr(ws),
                                      ctypes.c_void_p(s.cuda_stream))
    torch.cuda.current_stream(device).wait_stream(s)
    B.check(code, "ehl_newton_tvd")
    return dict(P=P, H0=H0, H=H, Hmin=Hmin, status=status, iters=iters)


def point_sweep_assemble(grid, params, P, Hel, H0, axis, color, opts=None):
    """Band systems of one colour of one sweep direction of the point
    contact (P, Hel: (B, Nx, Ny)).  Returns dict(band (B*lines, n, 9), rhs,
    bounded, direct (B, Nx, Ny))."""
    opts = opts or default_opts()
    for t, name in ((P, "P"), (Hel, "Hel"), (H0, "H0"), (params, "params")):
        _need(t, torch.float64, name)
    nb, Nx, Ny = P.shape
    nl, n = (Ny, Nx - 2) if axis == 0 else (Nx, Ny - 2)
    first = 1 if color == 1 else 2
    nlc = (nl - 2 - first) // 2 + 1 if first <= nl - 2 else 0
    dev = P.device
    band = torch.empty(nb * nlc, n, 9, dtype=torch.float64, device=dev)
    rhs = torch.empty(nb * nlc, n, dtype=torch.float64, device=dev)
    bounded = torch.empty(nb * nlc, n, dtype=torch.uint8, device=dev)
    direct = torch.empty(nb, Nx, Ny, dtype=torch.uint8, device=dev)
    ws = torch.empty(B.lib().ehl_point_assemble_workspace_bytes(ctypes.byref(grid), nb),
                     dtype=torch.uint8, device=dev)
    B.check(B.lib().ehl_point_sweep_assemble(handle(), ctypes.byref(grid), _ptr(params), nb,
                                             ctypes.byref(opts), int(axis), int(color), _ptr(P),
                                             _ptr(Hel), _ptr(H0), _ptr(band), _ptr(rhs),
                                             _ptr(bounded), _ptr(direct), _ptr(ws), _stream()),
            "ehl_point_sweep_assemble")
    return dict(band=band, rhs=rhs, bounded=bounded, direct=direct)


def solve_point(M, L, Nx, Ny, opts=None, P=None, H0=None, device=None, stream=None):
    """Alternating x/y line sweeps for B = len(M) point contacts on one grid
    (ehl_newton_tvd on a 2D grid).  The default options take the load
    relaxation c = 0.02: the 2D load responds about ten times more strongly to
    H0 than the line load, and c = 0.1 makes the H0 loop oscillate on 257 x 257
    nodes.  Returns dict(P (B, Nx, Ny), H0, H, Hmin, status, iters)."""
    opts = opts or default_opts(c_h0=0.02)
    device = device or torch.device("cuda", torch.cuda.current_device())
    grid = point_grid(Nx, Ny)
    params = params_tensor(M, L, device)
    nb = params.shape[0]
    P = torch.zeros(nb, Nx, Ny, dtype=torch.float64, device=device) if P is None else \
        P.clone().contiguous()
    H0 = torch.zeros(nb, dtype=torch.float64, device=device) if H0 is None else \
        torch.as_tensor(H0, dtype=torch.float64, device=device).clone()
    H = torch.empty(nb, Nx, Ny, dtype=torch.float64, device=device)
    Hmin = torch.empty(nb, dtype=torch.float64, device=device)
    status = torch.empty(nb, dtype=torch.int32, device=device)
    iters = torch.empty(nb, dtype=torch.int32, device=device)
    nbytes = B.lib().ehl_newton_workspace_bytes(handle(), ctypes.byref(grid), nb,
                                                ctypes.byref(opts))
    if nbytes == 0:
        raise ValueError("invalid EHL grid/options")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    s = stream or torch.cuda.Stream(device=device)
    s.wait_stream(torch.cuda.current_stream(device))
    with torch.cuda.stream(s):
        code = B.lib().ehl_newton_tvd(handle(), ctypes.byref(grid), _ptr(params), nb,
                                      ctypes.byref(opts), None, _ptr(P), _ptr(H0), _ptr(H),
                                      _ptr(Hmin), _ptr(status), _ptr(iters), _ptr(ws),
                                      ctypes.c_void_p(s.cuda_stream))
    torch.cuda.current_stream(device).wait_stream(s)
    B.check(code, "ehl_newton_tvd")
    return dict(P=P, H0=H0, H=H, Hmin=Hmin, status=status, iters=iters)


def adjoint(M, L, N, P, H0, gP=None, gH0=None, gH=None, rough=None, opts=None, rtol=1e-12,
            max_iter=400):
    """Gradients of a scalar output of converged line-contact solutions.

    (P, H0): the converged state, (B, N) and (B,).  gP, gH: (B, N) cotangents
    of the pressure and the film, gH0: (B,) of the offset (None = zero).
    Returns dict(dM, dL, drough, status, iters) as device tensors."""
    opts = opts or default_opts()
    _need(P, torch.float64, "P")
    _need(H0, torch.float64, "H0")
    nb = P.shape[0]
    dev = P.device
    for t, name in ((gP, "gP"), (gH0, "gH0"), (gH, "gH"), (rough, "rough")):
        if t is not None:
            _need(t, torch.float64, name)
    grid = line_grid(N)
    params = params_tensor(M, L, dev)
    dM = torch.empty(nb, dtype=torch.float64, device=dev)
    dL = torch.empty(nb, dtype=torch.float64, device=dev)
    drough = torch.empty(nb, N, dtype=torch.float64, device=dev)
    status = torch.empty(nb, dtype=torch.int32, device=dev)
    iters = torch.empty(nb, dtype=torch.int32, device=dev)
    nbytes = B.lib().ehl_adjoint_workspace_bytes(handle(), ctypes.byref(grid), nb)
    if nbytes == 0:
        raise ValueError("invalid EHL grid")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    B.check(B.lib().ehl_adjoint_solve(handle(), ctypes.byref(grid), _ptr(params), nb,
                                      ctypes.byref(opts), _ptr(rough), _ptr(P), _ptr(H0),
                                      _ptr(gP), _ptr(gH0), _ptr(gH), float(rtol), int(max_iter),
                                      _ptr(dM), _ptr(dL), _ptr(drough), _ptr(status),
                                      _ptr(iters), _ptr(ws), _stream()), "ehl_adjoint_solve")
    return dict(dM=dM, dL=dL, drough=drough, status=status, iters=iters)


class LineEHL(torch.autograd.Function):
    """Converged line-contact solve as a differentiable function.

    ``P, H0, H, status = LineEHL.apply(M, L, rough, N, opts)`` with M, L of
    shape (B,) and rough (B, N) or None; the backward pass is the hand-written
    adjoint (ehl_adjoint_solve) and gives gradients for M, L and rough.  An
    output such as Hmin = H.min(dim=1).values is differentiated by torch into
    the film cotangent at the arg-min.  The adjoint is the derivative of the
    converged fixed point: an instance whose forward solve did not converge
    (status not SYS_OK) gets NaN gradients."""

    @staticmethod
    def forward(ctx, M, L, rough, N, opts=None):
        ctx.set_materialize_grads(False)
        dev = rough.device if rough is not None else torch.device("cuda",
                                                                  torch.cuda.current_device())
        Mv = M.detach().to(torch.float64).cpu()
        Lv = L.detach().to(torch.float64).cpu()
        rg = None if rough is None else rough.detach().to(torch.float64).contiguous()
        r = solve_line(Mv, Lv, N, opts=opts, rough=rg, device=dev)
        ctx.save_for_backward(r["P"], r["H0"], r["status"])
        ctx.args = (Mv, Lv, rg, N, opts, M.device, L.device)
        ctx.mark_non_differentiable(r["status"])
        return r["P"], r["H0"], r["H"], r["status"]

    @staticmethod
    def backward(ctx, gP, gH0, gH, gstatus):
        P, H0, fst = ctx.saved_tensors
        Mv, Lv, rg, N, opts, mdev, ldev = ctx.args
        c = lambda t: None if t is None else t.to(torch.float64).contiguous()
        a = adjoint(Mv, Lv, N, P, H0, gP=c(gP), gH0=c(gH0), gH=c(gH), rough=rg, opts=opts)
        conv = fst == B.SYS_OK  # forward converged: the implicit-function adjoint holds
        bad = conv & (a["status"] != B.SYS_OK)
        if bad.any():
            raise RuntimeError(f"ehl_adjoint_solve: instance status {a['status'].tolist()}")
        nan = torch.tensor(float("nan"), dtype=torch.float64, device=P.device)
        dM = torch.where(conv, a["dM"], nan)
        dL = torch.where(conv, a["dL"], nan)
        drough = torch.where(conv[:, None], a["drough"], nan) if rg is not None else None
        return dM.to(mdev), dL.to(ldev), drough, None, None
