"""Pins of the oracle's exact adjoint (line contact).

  * the dense Jacobian of the residual with respect to the pressures (full log
    kernel) and to H0 against central finite differences of the residual map;
  * the adjoint gradients dH0/dM, dH0/dL, dHmin/dM, dHmin/dL and dHmin/droughness
    against central differences of re-converged solutions (step 1e-6
    relative), with the active set and arg-min checked unchanged;
  * with the kappa-scheme convection (kappa = 1/3): every pressurised column
    of the dense Jacobian against central differences (the slope is linear,
    so no branch switches), and dH0/dM, dHmin/dM, dH0/dL against central
    differences of re-converged kappa-scheme solutions.
"""
import numpy as np
import pytest

from oracle import deform
from oracle import ehl_adjoint as A
from oracle import ehl_line as E

N = 257


@pytest.fixture(scope="module")
def base():
    r = E.solve_line(20.0, 10.0, N)
    assert r["status"] == 0
    return r


def _branches(P, H0, x, kvec, ph, lam):
    """Limiter branch of every node (slopes of rho*H of the same sign)."""
    st = E.state(P, E.film(P, H0, x, kvec), ph, lam)
    rH = st["rH"]
    return (rH[1:-1] - rH[:-2]) * (rH[2:] - rH[1:-1]) > 0


def test_dense_jacobian_matches_residual_differences(base):
    r = base
    x, h, kvec = r["x"], r["h"], r["kvec"]
    _, lam, ph = E.moes_line(20.0, 10.0)
    P, H0 = r["P"], r["H0"]
    H = E.film(P, H0, x, kvec)
    RP, RH, _, _ = A.partials(P, H, ph, lam, h)
    K = deform.line_matrix(N, h)
    J = RP[:, 1:-1] + RH @ K[:, 1:-1]
    rng = np.random.default_rng(0)
    # pressurised columns only (the cavitated ones are not unknowns of the
    # adjoint, and the limiter is not differentiable where slopes vanish)
    inact = np.where(P[1:-1] > 0)[0]
    def fd_col(j, e):
        Pp, Pm = P.copy(), P.copy()
        Pp[j + 1] += e
        Pm[j + 1] -= e
        if (_branches(Pp, H0, x, kvec, ph, lam) != _branches(Pm, H0, x, kvec, ph, lam)).any():
            return None
        Rp, _ = E.residual(Pp, E.film(Pp, H0, x, kvec), ph, lam, h)
        Rm, _ = E.residual(Pm, E.film(Pm, H0, x, kvec), ph, lam, h)
        return (Rp - Rm) / (2 * e)

    checked = 0
    for j in rng.permutation(inact):
        # the van Leer limiter is not differentiable where a slope of rho*H
        # changes sign (extrema of rho*H) and its derivative varies fast next
        # to such points: use only columns where the branches do not switch and
        # two step sizes agree (the difference quotient is resolved)
        e = 1e-6 * max(1.0, abs(P[j + 1]))
        f1, f2 = fd_col(j, e), fd_col(j, e / 8)
        if f1 is None or f2 is None:
            continue
        sc = np.abs(f1[inact]).max()
        if np.abs(f1 - f2)[inact].max() > 1e-6 * sc:
            continue
        checked += 1
        assert np.abs(f2 - J[:, j])[inact].max() <= 1e-5 * sc + 1e-9, j
        if checked >= 12:
            break
    assert checked >= 6
    e = 1e-7
    Rp, _ = E.residual(P, E.film(P, H0 + e, x, kvec), ph, lam, h)
    Rm, _ = E.residual(P, E.film(P, H0 - e, x, kvec), ph, lam, h)
    fd = (Rp - Rm) / (2 * e)
    # rows of the pressurised nodes (the equations of the adjoint system)
    assert np.abs(fd - RH.sum(axis=1))[inact].max() <= 1e-5 * np.abs(fd[inact]).max()


def _solve(M, L, rough=None):
    r = E.solve_line(M, L, N, rough=rough)
    assert r["status"] == 0
    return r


def test_adjoint_parameters_vs_central_differences(base):
    M, L = 20.0, 10.0
    g = A.adjoint_gradients(base["P"], base["H0"], M, L, N)
    step = 1e-6
    rp, rm = _solve(M * (1 + step), L), _solve(M * (1 - step), L)
    assert (rp["P"][1:-1] > 0).tolist() == (rm["P"][1:-1] > 0).tolist()
    assert rp["argmin"] == rm["argmin"] == g["argmin"]
    fdH0 = (rp["H0"] - rm["H0"]) / (2 * step * M)
    fdHm = (rp["Hmin"] - rm["Hmin"]) / (2 * step * M)
    assert abs(fdH0 - g["dH0_dM"]) <= 1e-5 * abs(fdH0)
    assert abs(fdHm - g["dHmin_dM"]) <= 1e-5 * abs(fdHm)
    rp, rm = _solve(M, L * (1 + step)), _solve(M, L * (1 - step))
    fdH0 = (rp["H0"] - rm["H0"]) / (2 * step * L)
    fdHm = (rp["Hmin"] - rm["Hmin"]) / (2 * step * L)
    assert abs(fdH0 - g["dH0_dL"]) <= 1e-5 * abs(fdH0)
    assert abs(fdHm - g["dHmin_dL"]) <= 1e-5 * abs(fdHm)


def test_adjoint_roughness_vs_central_differences(base):
    M, L = 20.0, 10.0
    g = A.adjoint_gradients(base["P"], base["H0"], M, L, N)
    step = 1e-6
    for m in [g["argmin"], 120, 100]:
        rough = np.zeros(N)
        rough[m] = step
        rp = _solve(M, L, rough)
        rm = _solve(M, L, -rough)
        fd = (rp["Hmin"] - rm["Hmin"]) / (2 * step)
        assert abs(fd - g["dHmin_drough"][m]) <= 1e-5 * max(1.0, abs(fd)), (m, fd,
                                                                            g["dHmin_drough"][m])
        fd0 = (rp["H0"] - rm["H0"]) / (2 * step)
        assert abs(fd0 - g["dH0_drough"][m]) <= 1e-5 * max(1.0, abs(fd0))


KAPPA = 1.0 / 3.0


@pytest.fixture(scope="module")
def base_kappa():
    r = E.solve_line(20.0, 10.0, N, kappa=KAPPA)
    assert r["status"] == 0
    return r


def test_dense_jacobian_kappa_scheme(base_kappa):
    r = base_kappa
    x, h, kvec = r["x"], r["h"], r["kvec"]
    _, lam, ph = E.moes_line(20.0, 10.0)
    P, H0 = r["P"], r["H0"]
    RP, RH, _, _ = A.partials(P, E.film(P, H0, x, kvec), ph, lam, h, KAPPA)
    K = deform.line_matrix(N, h)
    J = RP[:, 1:-1] + RH @ K[:, 1:-1]
    inact = np.where(P[1:-1] > 0)[0]
    worst = 0.0
    for j in inact[::7]:
        e = 1e-6 * max(1.0, abs(P[j + 1]))
        Pp, Pm = P.copy(), P.copy()
        Pp[j + 1] += e
        Pm[j + 1] -= e
        Rp, _ = E.residual(Pp, E.film(Pp, H0, x, kvec), ph, lam, h, KAPPA)
        Rm, _ = E.residual(Pm, E.film(Pm, H0, x, kvec), ph, lam, h, KAPPA)
        fd = (Rp - Rm) / (2 * e)
        sc = np.abs(fd[inact]).max()
        worst = max(worst, np.abs(fd - J[:, j])[inact].max() / sc)
    assert worst <= 1e-5, worst


def test_adjoint_kappa_scheme_vs_central_differences(base_kappa):
    M, L = 20.0, 10.0
    g = A.adjoint_gradients(base_kappa["P"], base_kappa["H0"], M, L, N, kappa=KAPPA)
    step = 1e-6

    def solve(M_, L_):
        r = E.solve_line(M_, L_, N, kappa=KAPPA)
        assert r["status"] == 0
        return r

    rp, rm = solve(M * (1 + step), L), solve(M * (1 - step), L)
    assert (rp["P"][1:-1] > 0).tolist() == (rm["P"][1:-1] > 0).tolist()
    assert rp["argmin"] == rm["argmin"] == g["argmin"]
    fdH0 = (rp["H0"] - rm["H0"]) / (2 * step * M)
    fdHm = (rp["Hmin"] - rm["Hmin"]) / (2 * step * M)
    assert abs(fdH0 - g["dH0_dM"]) <= 1e-5 * abs(fdH0)
    assert abs(fdHm - g["dHmin_dM"]) <= 1e-5 * abs(fdHm)
    rp, rm = solve(M, L * (1 + step)), solve(M, L * (1 - step))
    fdH0 = (rp["H0"] - rm["H0"]) / (2 * step * L)
    assert abs(fdH0 - g["dH0_dL"]) <= 1e-5 * abs(fdH0)
