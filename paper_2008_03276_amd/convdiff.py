"""Linear convection-diffusion workload: binding of ``cd_example`` and
``cd_line_relax`` (argument marshalling only; the work runs in the HIP
library).  (a u)_x + (b u)_y - eps Lap u = f on [-1, 1]^2, kappa-scheme
convection, line relaxation with batched PAQIF line solves (defect correction,
the x-line splittings Ls0 / Ls1 and the distributive Ls3 splitting)."""
import ctypes

import torch

from . import _binding as B
from .paqif import _need, _ptr, _stream, handle


def example(n, eps=1e-6, a=1.0, b=1.0, device=None):
    """f for the exact solution x^4 + y^4 and the start iterate (exact
    boundary, zero inside), both (n, n) FP64 device tensors."""
    dev = torch.device("cuda") if device is None else torch.device(device)
    f = torch.empty((n, n), dtype=torch.float64, device=dev)
    u = torch.empty_like(f)
    B.check(B.lib().cd_example(int(n), float(eps), float(a), float(b), _ptr(f), _ptr(u),
                               _stream()), "cd_example")
    return f, u


def line_relax(f, u, kappa, eps=1e-6, a=1.0, b=1.0, omega=1.0, tol=1e-10, max_iter=500,
               workspace=None):
    """Run the line relaxation on u in place; returns (iterations, final max
    defect)."""
    _need(f, torch.float64, "f")
    _need(u, torch.float64, "u")
    n = int(u.shape[0])
    if tuple(u.shape) != (n, n) or tuple(f.shape) != (n, n):
        raise ValueError("f and u must be n x n")
    if workspace is None:
        workspace = torch.empty(max(1, B.lib().cd_workspace_bytes(n)), dtype=torch.uint8,
                                device=u.device)
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    B.check(B.lib().cd_line_relax(handle(), n, float(kappa), float(eps), float(a), float(b),
                                  float(omega), float(tol), int(max_iter), _ptr(f), _ptr(u),
                                  ctypes.byref(it), ctypes.byref(res), _ptr(workspace),
                                  _stream()), "cd_line_relax")
    return int(it.value), float(res.value)


def distributive_relax(f, u, kappa, eps=1e-6, a=1.0, b=1.0, omega=1.0, tol=1e-10, max_iter=500,
                       workspace=None):
    """Distributive line relaxation (Ls3) on u in place; returns
    (iterations, final max defect)."""
    _need(f, torch.float64, "f")
    _need(u, torch.float64, "u")
    n = int(u.shape[0])
    if tuple(u.shape) != (n, n) or tuple(f.shape) != (n, n):
        raise ValueError("f and u must be n x n")
    if workspace is None:
        workspace = torch.empty(max(1, B.lib().cd_ls3_workspace_bytes(n)), dtype=torch.uint8,
                                device=u.device)
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    B.check(B.lib().cd_distributive_relax(handle(), n, float(kappa), float(eps), float(a),
                                          float(b), float(omega), float(tol), int(max_iter),
                                          _ptr(f), _ptr(u), ctypes.byref(it), ctypes.byref(res),
                                          _ptr(workspace), _stream()), "cd_distributive_relax")
    return int(it.value), float(res.value)


def split_relax(f, u, which, kappa, eps=1e-6, a=1.0, b=1.0, omega=0.7, tol=1e-10, max_iter=500,
                workspace=None):
    """x-line splitting Ls0 (which = 0) or Ls1 (which = 1) on u in place;
    returns (iterations, final max defect)."""
    _need(f, torch.float64, "f")
    _need(u, torch.float64, "u")
    n = int(u.shape[0])
    if tuple(u.shape) != (n, n) or tuple(f.shape) != (n, n):
        raise ValueError("f and u must be n x n")
    if workspace is None:
        workspace = torch.empty(max(1, B.lib().cd_workspace_bytes(n)), dtype=torch.uint8,
                                device=u.device)
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    B.check(B.lib().cd_split_relax(handle(), n, int(which), float(kappa), float(eps), float(a),
                                   float(b), float(omega), float(tol), int(max_iter), _ptr(f),
                                   _ptr(u), ctypes.byref(it), ctypes.byref(res), _ptr(workspace),
                                   _stream()), "cd_split_relax")
    return int(it.value), float(res.value)
