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
    o = dict(omega=0.5, c_h0=0.1, switch_ratio=0.6, tol=1e-13, max_newton=4000, kernel_terms=1,
             lcp_max_iter=64, deform_prec=B.PREC_FP64, lcp_prec=B.PREC_FP64, steps_per_graph=16,
             start_rule=1)
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
