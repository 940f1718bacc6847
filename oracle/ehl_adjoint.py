"""Oracle (test infrastructure): exact adjoint of the converged line contact.

The converged state of the line-contact iteration (Sec. 3.3; see
ehl_line.py) satisfies, on the set I of interior nodes with P_i > 0,
    R_i(P, H0; theta) = 0,          i in I,
    G(P) = h sum_i P_i - pi/2 = 0   (load balance, eq. 75 at its fixed point),
with P_i = 0 on the cavitated nodes.  For an output J(P, H0; theta) (the
offset H0, or the minimum film Hmin = H_m* at its arg-min node m*) the
derivative with respect to a parameter theta, with the active set and m*
held fixed, is
    dJ/dtheta = dJ/dtheta|_explicit - lambda^T dF/dtheta,
    (dF/dy)^T lambda = dJ/dy,     y = (P_I, H0),  F = (R_I, G).
The Jacobian dF/dy is dense (every film value depends on every pressure
through the log kernel) and is assembled here exactly from the partial
derivatives of the discrete residual; the transposed system is solved with a
dense LU (library solve).  Parameters: M (through lam = 3 pi^2/(8 M^2) and
p_h proportional to sqrt(M)), L (p_h proportional to L) and the roughness
value R_m at every node (added to the film).

The paper has no adjoint; this is the exact derivative of its discrete
equations.  Pins: finite differences of the residual map (tests) and central
differences of re-converged solutions.
"""
import numpy as np

from . import deform
from . import ehl_line as E


def partials(P, H, ph, lam, h, kappa=None):
    """Dense partial derivatives of R_i (interior rows) with respect to the
    node pressures P_m (at fixed film), the node films H_m, lam and p_h
    (van Leer slope; with kappa given the kappa-scheme slope of ehl_line).

    Returns (RP, RH, Rlam, Rph): RP, RH of shape (N-2, N)."""
    N = len(P)
    n = N - 2
    st = E.state(P, H, ph, lam)
    rho, drho, dlneta, eps, rH = st["rho"], st["drho"], st["dlneta"], st["eps"], st["rH"]
    lam_eta = st["eta"] * lam
    eP = drho * H ** 3 / lam_eta - eps * dlneta      # d eps / dP at fixed H
    eH = 3.0 * rho * H ** 2 / lam_eta                 # d eps / dH
    dm = rH[1:-1] - rH[:-2]
    dp = rH[2:] - rH[1:-1]
    _, pa, pb = E.slope(dm, dp, kappa)                # index t -> node t+1
    Reps = np.zeros((n, N))
    RrH = np.zeros((n, N))
    Rp = np.zeros((n, N))
    for r in range(n):
        i = r + 1
        dPp = P[i + 1] - P[i]
        dPm = P[i] - P[i - 1]
        epsh_p = 0.5 * (eps[i] + eps[i + 1])
        epsh_m = 0.5 * (eps[i - 1] + eps[i])
        # diffusion: [eps_{i+1/2} dPp - eps_{i-1/2} dPm] / h^2
        Reps[r, i] += 0.5 * (dPp - dPm) / h ** 2
        Reps[r, i + 1] += 0.5 * dPp / h ** 2
        Reps[r, i - 1] += -0.5 * dPm / h ** 2
        Rp[r, i + 1] += epsh_p / h ** 2
        Rp[r, i] += -(epsh_p + epsh_m) / h ** 2
        Rp[r, i - 1] += epsh_m / h ** 2

        # flux: -(f_i - f_{i-1}) / h; f_t = rH_t + psi_t / 2 (t >= 1), f_0 = rH_0
        def add_flux(t, sign):
            if t == 0:
                RrH[r, 0] += sign
                return
            a_, b_ = pa[t - 1], pb[t - 1]
            RrH[r, t - 1] += sign * 0.5 * (-b_)
            RrH[r, t] += sign * (1.0 + 0.5 * (-a_ + b_))
            RrH[r, t + 1] += sign * 0.5 * a_

        add_flux(i, -1.0 / h)
        add_flux(i - 1, 1.0 / h)
    RP = Reps * eP[None, :] + RrH * (drho * H)[None, :] + Rp
    RH = Reps * eH[None, :] + RrH * rho[None, :]
    Rlam = Reps @ (-eps / lam)
    Rph = Reps @ (P / ph * eP) + RrH @ (P / ph * drho * H)
    return RP, RH, Rlam, Rph


def adjoint_gradients(P, H0, M, L, N, rough=None, kappa=None):
    """Gradients of H0 and Hmin at a converged state.

    Returns dict with dH0_dM, dH0_dL, dHmin_dM, dHmin_dL, dH0_drough (N),
    dHmin_drough (N), the inactive set and the arg-min node."""
    x, h = E.grid(N)
    K = deform.line_matrix(N, h)
    _, lam, ph = E.moes_line(M, L)
    H = E.film(P, H0, x, deform.line_kernel(N, h), rough)
    RP, RH, Rlam, Rph = partials(P, H, ph, lam, h, kappa)
    inact = np.where(P[1:-1] > 0.0)[0]           # rows r (node r+1) with P > 0
    cols = inact + 1                              # node indices
    nI = len(inact)
    # bordered Jacobian dF/dy, y = (P_I, H0)
    Jfull = RP[:, cols] + RH @ K[:, cols]
    cH = RH.sum(axis=1)
    A = np.zeros((nI + 1, nI + 1))
    A[:nI, :nI] = Jfull[inact]
    A[:nI, nI] = cH[inact]
    A[nI, :nI] = h
    # parameter derivatives of F (load row has none)
    dlam_dM = -2.0 * lam / M
    dph_dM = ph / (2.0 * M)
    dph_dL = ph / L
    FM = np.concatenate([(Rlam * dlam_dM + Rph * dph_dM)[inact], [0.0]])
    FL = np.concatenate([(Rph * dph_dL)[inact], [0.0]])
    Frough = np.vstack([RH[inact], np.zeros((1, N))])      # (nI+1) x N
    mstar = int(np.argmin(H))
    out = dict(inactive=cols, argmin=mstar)
    for name, g, dexp_rough in (
            ("H0", np.concatenate([np.zeros(nI), [1.0]]), np.zeros(N)),
            ("Hmin", np.concatenate([K[mstar, cols], [1.0]]), np.eye(N)[mstar])):
        lamv = np.linalg.solve(A.T, g)
        out[f"d{name}_dM"] = -lamv @ FM
        out[f"d{name}_dL"] = -lamv @ FL
        out[f"d{name}_drough"] = dexp_rough - lamv @ Frough
    return out
