"""Pins of the line-contact physics of the oracle against facts outside it.

Each test fixes one oracle function by something the oracle does not
compute itself: the dimensional definitions behind the Moes parameters
(appendix), closed-form values and limits of the Roelands and
Dowson-Higginson laws (Sec. 3.3, line-contact example), the textbook ratio
form of the van Leer limiter, exact differences on polynomial fields, an
independent quadrature solution of the rigid-isoviscous problem, the
Hertzian dry-contact limit at high load, and the observed grid order of the
paper's error norms (eqs. 96-97).
"""
import warnings

import numpy as np
import pytest

from oracle import ehl_line as E


# ---------------------------------------------------------------------------
# Moes map (appendix): from dimensional definitions
# ---------------------------------------------------------------------------

def test_moes_line_map_from_dimensional_definitions():
    """alpha_bar, lambda_bar and p_h of the oracle against a dimensional
    line contact: W = w/(E'R), 2U = eta0 u_s/(E'R), G = alpha E',
    M = W (2U)^(-1/2), L = G (2U)^(1/4) (appendix); Hertzian half-width
    b = sqrt(8 w R/(pi E')) and peak pressure p_h = 2 w/(pi b) of a loaded
    cylinder; lambda = 6 eta0 u_s R^2/(b^3 p_h) (Sec. 3.3)."""
    for Ep, R, w, eta0, us in [(2.2e11, 0.01, 1.0e5, 0.05, 2.0),
                               (1.1e11, 0.02, 4.0e5, 0.4, 0.5),
                               (2.3e11, 0.005, 2.5e4, 0.01, 10.0)]:
        alpha = E.ALPHA
        W = w / (Ep * R)
        twoU = eta0 * us / (Ep * R)
        G = alpha * Ep
        M = W * twoU ** -0.5
        L = G * twoU ** 0.25
        b = np.sqrt(8.0 * w * R / (np.pi * Ep))
        ph = 2.0 * w / (np.pi * b)
        lam = 6.0 * eta0 * us * R * R / (b ** 3 * ph)
        abar_o, lam_o, ph_o = E.moes_line(M, L)
        assert abs(abar_o - alpha * ph) <= 1e-12 * alpha * ph
        assert abs(lam_o - lam) <= 1e-12 * lam
        assert abs(ph_o - ph) <= 1e-12 * ph
        # the dimensionless load pi/2 is the dimensional load w
        assert abs(ph * b * np.pi / 2.0 - w) <= 1e-12 * w


# ---------------------------------------------------------------------------
# Lubricant laws (Sec. 3.3): Roelands viscosity, Dowson-Higginson density
# ---------------------------------------------------------------------------

def test_lubricant_closed_forms():
    ph = 5.0e8
    P = np.array([0.0, 0.59e9 / ph, E.P0_ROELANDS / ph, 1e6])
    rho, drho, lneta, dlneta = E.lubricant(P, ph)
    # density: 1 at ambient pressure, 2.34/2 at p = 0.59 GPa, -> 1.34
    assert rho[0] == 1.0
    assert abs(rho[1] - 1.17) <= 1e-15
    assert abs(rho[3] - 1.34) < 1e-6 and rho[3] < 1.34
    # viscosity: ln eta = 0 at ambient pressure; at p = p0 it is
    # (alpha p0 / z)(2^z - 1) = (3.366 / 0.68)(2^0.68 - 1), by hand
    # 2^0.68 = exp(0.68 ln 2) = exp(0.47134008) = 1.60213976, so
    # 4.95 * 0.60213976 = 2.98059179
    assert lneta[0] == 0.0
    assert abs(lneta[2] - 2.98059179) < 5e-8
    # Roelands reduces to Barus at low pressure: d ln eta / dp = alpha,
    # i.e. d ln eta / dP = alpha p_h at P = 0
    assert abs(dlneta[0] - E.ALPHA * ph) <= 1e-14 * E.ALPHA * ph
    # and the low-pressure density slope of Dowson-Higginson:
    # d rho/dp = (1.34 - 1)/0.59e9 at p = 0
    assert abs(drho[0] - 0.34 / 0.59e9 * ph) <= 1e-14 * ph


def test_lubricant_derivatives_match_differences():
    ph = 4.0e8
    P = np.linspace(0.0, 3.0, 13)
    rho, drho, lneta, dlneta = E.lubricant(P, ph)
    d = 1e-6
    rp, _, lp, _ = E.lubricant(P + d, ph)
    rm, _, lm, _ = E.lubricant(P - d, ph)
    assert np.abs((rp - rm) / (2 * d) - drho).max() <= 1e-8 * np.abs(drho).max()
    assert np.abs((lp - lm) / (2 * d) - dlneta).max() <= 1e-8 * np.abs(dlneta).max()
    # monotone: both grow with pressure
    assert (np.diff(rho) > 0).all() and (np.diff(lneta) > 0).all()


# ---------------------------------------------------------------------------
# Limiter (the paper does not name it; van Leer is the reading)
# ---------------------------------------------------------------------------

def _vanleer_ratio_form(dm, dp):
    """Textbook van Leer: psi = phi(r) D-, r = D+/D-, phi(r) = (r + |r|)/(1 + |r|)."""
    out = np.zeros_like(dm)
    nz = dm != 0.0
    r = dp[nz] / dm[nz]
    out[nz] = (r + np.abs(r)) / (1.0 + np.abs(r)) * dm[nz]
    return out


def test_vanleer_properties():
    rng = np.random.default_rng(5)
    dm = rng.normal(size=2000)
    dp = rng.normal(size=2000)
    psi, pa, pb = E.vanleer(dm, dp)
    # the textbook ratio form
    assert np.abs(psi - _vanleer_ratio_form(dm, dp)).max() <= 1e-14 * np.abs(psi).max()
    # linear data: the common slope
    d = rng.normal(size=50)
    assert np.abs(E.vanleer(d, d)[0] - d).max() <= 1e-15 * np.abs(d).max()
    # extrema: zero
    ext = dm * dp <= 0
    assert (psi[ext] == 0.0).all()
    # TVD region: between 0 and twice either difference, same sign
    same = ~ext
    assert (psi[same] / dm[same] >= 0).all() and (psi[same] / dm[same] <= 2.0 + 1e-15).all()
    assert (psi[same] / dp[same] >= 0).all() and (psi[same] / dp[same] <= 2.0 + 1e-15).all()
    # symmetric in its two arguments
    assert np.abs(E.vanleer(dp, dm)[0] - psi).max() <= 1e-15 * np.abs(psi).max()
    # partials against central differences (away from the kink)
    h = 1e-7
    far = same & (np.abs(dm) > 1e-2) & (np.abs(dp) > 1e-2)
    fd_p = (E.vanleer(dm, dp + h)[0] - E.vanleer(dm, dp - h)[0]) / (2 * h)
    fd_m = (E.vanleer(dm + h, dp)[0] - E.vanleer(dm - h, dp)[0]) / (2 * h)
    assert np.abs(fd_p - pa)[far].max() < 1e-6
    assert np.abs(fd_m - pb)[far].max() < 1e-6


# ---------------------------------------------------------------------------
# Residual (eqs. 62-65, line form): exact on polynomial fields, second order
# ---------------------------------------------------------------------------

def test_residual_convective_part_exact_on_linear_film():
    """P = 0 and p_h = 0 (rho = eta = 1): R = -(flux difference)/h; on a
    linear film the limited face values are exact, so R_i = -H' for every
    row with two upstream neighbours; the inlet row sees the first-order
    inlet face (psi_0 = 0) and gets -3/2 H'."""
    N = 41
    x, h = E.grid(N)
    for slope in (0.7, -0.3):
        H = 2.0 + slope * (x - x[0])
        R, _ = E.residual(np.zeros(N), H, 0.0, 1.0, h)
        assert np.abs(R[1:] + slope).max() <= 1e-12
        assert abs(R[0] + 1.5 * slope) <= 1e-12


def test_residual_diffusive_part_exact_on_quadratic_pressure():
    """rho H constant (no convection), eps = H^3/lam = 1: R_i = P''(X_i)
    exactly for a quadratic P."""
    N = 33
    x, h = E.grid(N)
    P = 0.4 + 0.3 * x + 1.25 * x * x
    R, _ = E.residual(P, np.ones(N), 0.0, 1.0, h)
    assert np.abs(R - 2.5).max() <= 1e-9


def test_residual_second_order_on_smooth_fields():
    """Smooth monotone film and smooth pressure (rho = eta = 1, lam = 1):
    R_i -> (H^3 P')' - H' at second order (rows past the inlet row)."""
    def fields(N):
        x, h = E.grid(N)
        H = 1.0 + 0.1 * (x + 4.5)
        P = np.sin(0.5 * x) + 2.0
        exact = (3 * H * H * 0.1 * 0.5 * np.cos(0.5 * x) - H ** 3 * 0.25 * np.sin(0.5 * x)) - 0.1
        R, _ = E.residual(P, H, 0.0, 1.0, h)
        return np.abs(R[1:] - exact[2:-1]).max()
    e = [fields(N) for N in (65, 129, 257)]
    assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5, e


# ---------------------------------------------------------------------------
# Rigid-isoviscous limit: independent quadrature shoot of the Reynolds ODE
# ---------------------------------------------------------------------------

def _rigid_isoviscous_reference(M):
    """K = 0, rho = eta = 1: H = H0 + X^2/2; integrating the Reynolds
    equation once with the Reynolds exit condition P = P' = 0 at Xc gives
    P'(X) = lam (H - H(Xc)) / H^3 (lam = 3 pi^2/(8 M^2)), P(-4.5) = 0,
    P(Xc) = 0, load integral pi/2.  Solved by nested root finding on
    adaptive quadratures (scipy), nothing from the oracle."""
    from scipy import integrate, optimize
    lam = 3.0 * np.pi ** 2 / (8.0 * M * M)
    xa = E.XA

    def g(t, H0, Hm):
        H = H0 + 0.5 * t * t
        return (H - Hm) / H ** 3

    def exit_and_load(H0):
        F = lambda xc: integrate.quad(g, xa, xc, args=(H0, H0 + 0.5 * xc * xc),
                                      epsabs=1e-15, epsrel=1e-14, limit=200)[0]
        xc = optimize.brentq(F, 1e-9, 1.5, xtol=1e-15)
        Hm = H0 + 0.5 * xc * xc
        load = lam * integrate.quad(lambda t: (xc - t) * g(t, H0, Hm), xa, xc,
                                    epsabs=1e-15, epsrel=1e-14, limit=200)[0]
        return xc, Hm, load

    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        H0 = optimize.brentq(lambda v: exit_and_load(v)[2] - np.pi / 2.0, 1e-4, 1.0, xtol=1e-15)
        xc, Hm, _ = exit_and_load(H0)

        def pressure(x):
            if x >= xc:
                return 0.0
            return lam * integrate.quad(g, xa, x, args=(H0, Hm), epsabs=1e-15, epsrel=1e-13,
                                        limit=200)[0]
        return H0, xc, pressure


def test_rigid_isoviscous_limit_against_ode_shoot():
    M = 3.0
    H0_ref, xc, pressure = _rigid_isoviscous_reference(M)
    errs_h0, errs_p = [], []
    for N in (129, 257, 513):
        r = E.solve_line(M, 0.0, N, rigid=True)
        assert r["status"] == 0
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            Pref = np.array([pressure(v) for v in r["x"]])
        errs_h0.append(abs(r["H0"] - H0_ref) / H0_ref)
        errs_p.append(np.abs(r["P"] - Pref).max() / Pref.max())
    # close to the continuous solution and converging under refinement
    assert errs_h0[-1] < 1e-3 and errs_p[-1] < 1e-3, (errs_h0, errs_p)
    assert errs_h0[0] / errs_h0[1] > 2.5 and errs_h0[1] / errs_h0[2] > 2.5, errs_h0
    assert errs_p[0] / errs_p[1] > 2.5 and errs_p[1] / errs_p[2] > 2.5, errs_p


# ---------------------------------------------------------------------------
# Hertzian limit: the pressure tends to sqrt(1 - X^2) as the load grows
# ---------------------------------------------------------------------------

def test_hertzian_limit_as_load_grows():
    """M in {20, 100, 200} at L = 10 on 513 nodes (M >= 500 needs a finer
    grid: its film falls below the mesh width and the iteration does not
    converge there).  The distance to the Hertzian pressure falls strictly
    and the film flattens inside the contact."""
    dist, flat = [], []
    for M in (20.0, 100.0, 200.0):
        r = E.solve_line(M, 10.0, 513)
        assert r["status"] == 0
        x = r["x"]
        herz = np.sqrt(np.clip(1.0 - x * x, 0.0, None))
        dist.append(np.sqrt(r["h"] * ((r["P"] - herz) ** 2).sum()))
        Hin = r["H"][np.abs(x) < 0.9]
        flat.append((Hin.max() - Hin.min()) / Hin.mean())
    assert dist[0] > dist[1] > dist[2], dist
    assert dist[2] < 0.2 * dist[0]
    assert flat[0] > flat[1] > flat[2], flat


# ---------------------------------------------------------------------------
# Grid order with the paper's error norms (eqs. 96-97)
# ---------------------------------------------------------------------------

def _norms(coarse, fine, hc):
    d = coarse - fine[::2]   # injection of the fine solution into the coarse nodes
    return np.sqrt(hc * (d * d).sum()), hc * np.abs(d).sum()


def test_observed_grid_order_eqs_96_97():
    """L2(k, k-1) = sqrt(H sum (u~^{k-1} - I u^k)^2) between consecutive
    grids and p2 = log2(L2(k-1, k-2) / L2(k, k-1)) (eq. 97), for M = 10,
    L = 5 on 65, 129, 257 and 513 nodes: the film converges at second order
    (the TVD scheme is second order away from extrema and the free
    boundary), the pressure, with its spike, at least at first order."""
    sols = {N: E.solve_line(10.0, 5.0, N) for N in (65, 129, 257, 513)}
    assert all(s["status"] == 0 for s in sols.values())
    Ns = sorted(sols)
    nH = [_norms(sols[a]["H"], sols[b]["H"], sols[a]["h"]) for a, b in zip(Ns[:-1], Ns[1:])]
    nP = [_norms(sols[a]["P"], sols[b]["P"], sols[a]["h"]) for a, b in zip(Ns[:-1], Ns[1:])]
    pH2 = [np.log2(a[0] / b[0]) for a, b in zip(nH[:-1], nH[1:])]
    pH1 = [np.log2(a[1] / b[1]) for a, b in zip(nH[:-1], nH[1:])]
    pP1 = np.log2(nP[-2][1] / nP[-1][1])
    assert min(pH2) > 1.8 and min(pH1) > 1.8, (pH2, pH1)
    assert pP1 > 1.5, pP1
