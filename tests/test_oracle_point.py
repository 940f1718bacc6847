"""Pins of the point-contact oracle (CPU).

  * Moes point-contact map against the dimensional definitions (Hertz
    radius a^3 = 3FR/(2E'), p_h = 3F/(2 pi a^2), lam = 6 eta0 u_s R^2 /
    (a^3 p_h), M = W (2U)^(-3/4), L = G (2U)^(1/4));
  * the line Jacobians of both sweep directions against finite differences of
    the 2D residual where the line model is exact (rigid film, all nodes
    direct), with the van Leer slope and with the kappa-scheme (kappa = 0,
    1/3, -1);
  * the 2D residual in flux form: its sum over the interior telescopes to the
    boundary fluxes;
  * the weighted change of eq. 69 conserves the change of an interior
    distributive node (sigma - 4 sigma/4 = 0);
  * the converged 33 x 33 contact (van Leer, and the kappa-scheme with
    kappa = 1/3): complementarity, load balance 2 pi/3, y-mirror symmetry,
    positive film;
  * the Lhs1 / Lhs2 line matrices of both sweep directions against finite
    differences of their implicit operator (elastic film, weighted changes),
    and the Lhs2 iteration's fixed point equal to the Newton iteration's.
"""
import numpy as np
import pytest

from oracle import deform
from oracle import ehl_line as OL
from oracle import ehl_point as OP


def test_moes_point_map_from_dimensional_definitions():
    Ep, R, F, eta0, us, alpha = 2.2e11, 0.02, 500.0, 0.04, 2.0, OL.ALPHA
    W = F / (Ep * R * R)
    U2 = eta0 * us / (Ep * R)
    G = alpha * Ep
    M = W * U2 ** -0.75
    L = G * U2 ** 0.25
    a = (3.0 * F * R / (2.0 * Ep)) ** (1.0 / 3.0)
    ph = 3.0 * F / (2.0 * np.pi * a * a)
    lam = 6.0 * eta0 * us * R * R / (a ** 3 * ph)
    abar, lam_o, ph_o = OP.moes_point(M, L)
    assert abs(abar - alpha * ph) <= 1e-12 * abar
    assert abs(ph_o - ph) <= 1e-12 * ph
    assert abs(lam_o - lam) <= 1e-12 * lam


def _rigid_state(Nx, Ny, M=20.0, seed=0):
    X, Y, hx, hy = OP.grid(Nx, Ny)
    rng = np.random.default_rng(seed)
    P = OP.hertz_start(X, Y) * (1 + 0.3 * rng.random((Nx, Ny)))
    P[0, :] = P[-1, :] = P[:, 0] = P[:, -1] = 0.0
    H = 0.3 + 0.5 * X[:, None] ** 2 + 0.5 * Y[None, :] ** 2 + 0.05 * rng.random((Nx, Ny))
    _, lam, ph = OP.moes_point(M, 10.0)
    return X, Y, hx, hy, P, H, lam, ph


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("kappa", [None, 0.0, 1.0 / 3.0, -1.0])
def test_line_jacobian_matches_finite_differences_rigid_direct(axis, kappa):
    Nx, Ny = 15, 11
    X, Y, hx, hy, P, H, lam, ph = _rigid_state(Nx, Ny)
    st = OL.state(P, H, ph, lam)
    direct = np.ones((Nx, Ny), dtype=bool)
    k2 = np.zeros((Nx, Ny))                       # rigid film: H does not move
    A, _, _ = OP.sweep_systems(P, H, st, ph, lam, hx, hy, k2, direct, axis, 2, limjac=0,
                               kappa=kappa)
    nl, nn = (Ny, Nx) if axis == 0 else (Nx, Ny)
    e = 1e-7
    worst = 0.0
    for l in range(1, nl - 1):
        for k in range(1, nn - 1):
            node = (k, l) if axis == 0 else (l, k)
            Pp, Pm = P.copy(), P.copy()
            Pp[node] += e
            Pm[node] -= e
            Rp, _ = OP.residual(Pp, H, ph, lam, hx, hy, kappa)
            Rm, _ = OP.residual(Pm, H, ph, lam, hx, hy, kappa)
            col = (Rp - Rm) / (2 * e)
            col_line = col[:, l - 1] if axis == 0 else col[l - 1, :]
            for s in range(-4, 5):
                r = k - 1 - s
                if 0 <= r < nn - 2:
                    ref = col_line[r]
                    worst = max(worst, abs(-A[l - 1, r, s + 4] - ref) /
                                max(1.0, np.abs(col_line).max()))
            # the line system has no coupling to other lines' unknowns
    assert worst <= 1e-6, worst


def test_residual_flux_form_telescopes():
    Nx, Ny = 21, 17
    X, Y, hx, hy, P, H, lam, ph = _rigid_state(Nx, Ny, seed=3)
    R, st = OP.residual(P, H, ph, lam, hx, hy)
    eps, rH = st["eps"], st["rH"]
    ex = 0.5 * (eps[:-1, :] + eps[1:, :])
    ey = 0.5 * (eps[:, :-1] + eps[:, 1:])
    f, _, _ = OP.x_flux(rH)
    js = slice(1, Ny - 1)
    is_ = slice(1, Nx - 1)
    bx = (ex[-1, js] * (P[-1, js] - P[-2, js]) - ex[0, js] * (P[1, js] - P[0, js])).sum() / hx ** 2
    by = (ey[is_, -1] * (P[is_, -1] - P[is_, -2]) - ey[is_, 0] * (P[is_, 1] - P[is_, 0])).sum() / hy ** 2
    bc = (f[-1, js] - f[0, js]).sum() / hx
    total = bx + by - bc
    assert abs(R.sum() - total) <= 1e-10 * np.abs(R).sum()


def test_weighted_change_conserves_interior_change():
    N = 9
    P = np.ones((N, N))
    P[0, :] = P[-1, :] = P[:, 0] = P[:, -1] = 0.0
    direct = np.zeros((N, N), dtype=bool)
    direct[0, :] = direct[-1, :] = direct[:, 0] = direct[:, -1] = True
    sig = np.zeros((N, N))
    sig[4, 4] = 0.3
    Pn = OP.sweep_update(P, sig, direct, 1.0)
    d = Pn - P
    assert abs(d.sum()) <= 1e-15
    assert d[4, 4] == pytest.approx(0.3) and d[3, 4] == pytest.approx(-0.075)
    direct[4, 4] = True
    Pn = OP.sweep_update(P, sig, direct, 1.0)
    d = Pn - P
    assert d[4, 4] == pytest.approx(0.3) and np.count_nonzero(d) == 1


@pytest.fixture(scope="module")
def converged():
    r = OP.solve_point(20.0, 10.0, 33, 33, tol=1e-11, max_steps=1200)
    assert r["status"] == 0
    return r


def test_converged_point_contact(converged):
    r = converged
    P, H, hx, hy = r["P"], r["H"], r["hx"], r["hy"]
    _, lam, ph = OP.moes_point(20.0, 10.0)
    R, st = OP.residual(P, H, ph, lam, hx, hy)
    Pi = P[1:-1, 1:-1]
    scale = np.abs(st["rH"]).max() / hx
    press = Pi > 1e-8
    assert (P >= 0).all()
    assert np.abs(R[press]).max() <= 1e-6 * scale
    assert (-R[~press] >= -1e-6 * scale).all()
    assert abs(hx * hy * P.sum() - OP.LOAD) <= 1e-10
    assert np.abs(P - P[:, ::-1]).max() <= 1e-12
    assert H.min() > 0
    # the pressure maximum lies inside the Hertzian circle and is of
    # Hertzian size (the outlet lobes of EHL can exceed the centre value)
    i, j = np.unravel_index(np.argmax(P), P.shape)
    assert r["X"][i] ** 2 + r["Y"][j] ** 2 < 1.0 and 0.8 < P.max() < 1.5


def test_converged_point_contact_kappa_scheme():
    # kappa = 1/3: complementarity of the kappa-scheme residual, load balance,
    # y-mirror symmetry and a positive film, like the van Leer contact
    k = 1.0 / 3.0
    r = OP.solve_point(20.0, 10.0, 33, 33, tol=1e-11, max_steps=1200, kappa=k)
    assert r["status"] == 0
    P, H, hx, hy = r["P"], r["H"], r["hx"], r["hy"]
    _, lam, ph = OP.moes_point(20.0, 10.0)
    R, st = OP.residual(P, H, ph, lam, hx, hy, k)
    Pi = P[1:-1, 1:-1]
    scale = np.abs(st["rH"]).max() / hx
    press = Pi > 1e-8
    assert (P >= 0).all()
    assert np.abs(R[press]).max() <= 1e-6 * scale
    assert (-R[~press] >= -1e-6 * scale).all()
    assert abs(hx * hy * P.sum() - OP.LOAD) <= 1e-10
    assert np.abs(P - P[:, ::-1]).max() <= 1e-12
    assert H.min() > 0


def _point_implicit(sig, l, axis, P, H, eps, rho, hx, hy, k2, direct, kterms, c):
    """Implicit operator of the splitting Lhs1 / Lhs2 on line l as a function
    of that line's changes sig (interior positions), from eqs. 62 and 69-74:
    eps and rho at the current iterate; the change field delta = D sigma
    (sigma at the node, -sigma/4 to the four neighbours of a weighted-change
    node); the film moves by the 2D kernel sum of each column's change field,
    kept where the along-line offset to the column is at most kterms; the
    x-convection is the upwind rho H weighted by c.  Returns the rows of the
    line's interior nodes."""
    Nx, Ny = P.shape
    node = (lambda ll, m: (m, ll)) if axis == 0 else (lambda ll, m: (ll, m))
    nn = Nx if axis == 0 else Ny
    Pb, Hb = P.copy(), H.copy()
    ii, jj = np.meshgrid(np.arange(Nx), np.arange(Ny), indexing="ij")
    along = ii if axis == 0 else jj
    for k in range(1, nn - 1):
        if sig[k - 1] == 0.0:
            continue
        d = np.zeros_like(P)
        i0, j0 = node(l, k)
        d[i0, j0] = 1.0
        if not direct[i0, j0]:
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                a, b = i0 + di, j0 + dj
                if 1 <= a <= Nx - 2 and 1 <= b <= Ny - 2:
                    d[a, b] -= 0.25
        resp = np.zeros_like(P)
        for a, b in zip(*np.nonzero(d)):
            resp += d[a, b] * k2[np.abs(ii - a), np.abs(jj - b)]
        Pb += sig[k - 1] * d
        Hb += sig[k - 1] * np.where(np.abs(along - k) <= kterms, resp, 0.0)
    ex = 0.5 * (eps[1:, :] + eps[:-1, :])
    ey = 0.5 * (eps[:, 1:] + eps[:, :-1])
    f = rho * Hb
    out = []
    for m in range(1, nn - 1):
        i, j = node(l, m)
        r = (ex[i, j] * (Pb[i + 1, j] - Pb[i, j]) - ex[i - 1, j] * (Pb[i, j] - Pb[i - 1, j])) / hx ** 2
        r += (ey[i, j] * (Pb[i, j + 1] - Pb[i, j]) - ey[i, j - 1] * (Pb[i, j] - Pb[i, j - 1])) / hy ** 2
        r -= c * (f[i, j] - f[i - 1, j]) / hx
        out.append(r)
    return np.array(out)


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("split,kappa", [(1, None), (2, None), (2, 1.0 / 3.0)])
def test_splitting_line_matrix_matches_finite_differences(axis, split, kappa):
    """The point contact's Lhs1 / Lhs2 line matrices are the derivatives of
    the implicit operator above (elastic film, weighted-change nodes; y-lines:
    the rows of direct nodes, the others stay identity rows)."""
    Nx, Ny, kterms, l = 13, 11, 2, 5
    X, Y, hx, hy, P, H, lam, ph = _rigid_state(Nx, Ny, seed=4)
    st = OL.state(P, H, ph, lam)
    rng = np.random.default_rng(8)
    direct = rng.random((Nx, Ny)) < 0.5
    direct[0, :] = direct[-1, :] = direct[:, 0] = direct[:, -1] = True
    k2 = deform.point_kernel(Nx, Ny, hx, hy)
    A, _, _ = OP.sweep_systems(P, H, st, ph, lam, hx, hy, k2, direct, axis, kterms,
                               kappa=kappa, split=split)
    kk = 0.0 if kappa is None else kappa
    c = (2 - kk) / 2 if split == 1 else (2 - kk) / 2 + (1 - kk) / 4
    nn = Nx if axis == 0 else Ny
    n = nn - 2
    e = 1e-6
    Jfd = np.zeros((n, n))
    for k in range(n):
        s = np.zeros(n)
        s[k] = e
        Jfd[:, k] = (_point_implicit(s, l, axis, P, H, st["eps"], st["rho"], hx, hy, k2, direct,
                                     kterms, c) -
                     _point_implicit(-s, l, axis, P, H, st["eps"], st["rho"], hx, hy, k2, direct,
                                     kterms, c)) / (2 * e)
    Ad = np.zeros((n, n))
    for r in range(n):
        for s in range(-4, 5):
            if 0 <= r + s < n:
                Ad[r, r + s] = A[l - 1, r, s + 4]
    rows = np.arange(n)
    if axis == 1:
        rows = rows[direct[l, 1:-1]]
        frozen = ~direct[l, 1:-1]
        assert (Ad[frozen] == np.eye(n)[frozen]).all()
    err = np.abs(-Ad[rows] - Jfd[rows]).max()
    assert err <= 1e-9 * np.abs(Jfd[rows]).max(), err
    An, _, _ = OP.sweep_systems(P, H, st, ph, lam, hx, hy, k2, direct, axis, kterms, limjac=0,
                                kappa=kappa)
    assert np.abs(An[l - 1] - A[l - 1]).max() > 1e3 * err


def test_splitting_reaches_the_newton_fixed_point_point_contact():
    """Lhs2 on the 17 x 17 contact converges to the Newton iteration's fixed
    point (the splitting changes the iteration, not the equations)."""
    ref = OP.solve_point(20.0, 10.0, 17, 17, tol=1e-13, max_steps=1500)
    r = OP.solve_point(20.0, 10.0, 17, 17, tol=1e-13, max_steps=1500, splitting=2)
    assert ref["status"] == 0 and r["status"] == 0
    assert np.abs(r["P"] - ref["P"]).max() <= 1e-10 * np.abs(ref["P"]).max()
    assert abs(r["H0"] - ref["H0"]) <= 1e-10 * abs(ref["H0"])
