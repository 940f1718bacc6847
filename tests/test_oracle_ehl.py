"""Pins of the oracle's deformation kernels and EHL line-contact pieces.

  * cell integrals of the log kernel and of the point (1/r) kernel against
    numerical quadrature; symmetry;
  * Hertz identities: with the Hertzian pressure, X^2/2 + H_el is constant
    inside the contact (line: 1/4 + ln2/2; point: 1), and the discrete
    versions converge to it under refinement;
  * the direct 2D sum against a plain quadruple loop;
  * the band Jacobian against central finite differences of the residual
    (with the film map the Jacobian claims to linearise);
  * the converged line contact (M=20, L=10, N=257): complementarity, load
    balance, the flux invariant of the Reynolds equation, positivity of H;
  * the Lhs1 / Lhs2 splitting matrices against finite differences of their
    implicit operator (eps, rho frozen; weighted upwind convection), and the
    fixed point of those iterations equal to the Newton iteration's.
"""
import numpy as np
import pytest
import scipy.integrate as si

from oracle import deform
from oracle import ehl_line as E


def test_line_cell_integral_quadrature():
    h = 0.05
    for d in [0.0, 0.01, 0.025, 0.03, 0.1, -0.1, 1.7, -3.3]:
        ref = si.quad(lambda t: np.log(abs(t)), d - h / 2, d + h / 2,
                      points=[0.0] if abs(d) <= h / 2 else None, limit=200)[0]
        got = deform.line_cell_integral(np.array([d]), h)[0]
        assert abs(got - ref) < 1e-13, (d, got, ref)
    # symmetry and self term h (ln(h/2) - 1)
    assert np.allclose(deform.line_cell_integral(np.array([0.3]), h),
                       deform.line_cell_integral(np.array([-0.3]), h), rtol=0, atol=1e-16)
    assert abs(deform.line_cell_integral(np.array([0.0]), h)[0] - h * (np.log(h / 2) - 1)) < 1e-15


def test_line_hertz_identity_converges():
    errs = []
    for N in [129, 513, 2049]:
        x, h = E.grid(N)
        P = E.hertz_start(x)
        Hel = deform.line_deformation(P, h)
        g = 0.5 * x * x + Hel
        inside = np.abs(x) < 0.8
        target = 0.25 + 0.5 * np.log(2.0)
        errs.append(np.abs(g[inside] - target).max())
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 2e-3


def test_point_cell_integral_quadrature():
    hx = hy = 0.1
    for dx, dy in [(0.1, 0.0), (0.2, -0.3), (-0.07, 0.09), (1.0, 0.7)]:
        f = lambda yp, xp: 1.0 / np.hypot(dx - xp, dy - yp)
        ref = si.dblquad(f, -hx / 2, hx / 2, -hy / 2, hy / 2, epsabs=1e-13, epsrel=1e-12)[0]
        got = deform.point_cell_integral(np.array(dx), np.array(dy), hx, hy)
        assert abs(float(got) - ref) < 1e-9 * max(1, ref), (dx, dy, got, ref)
    self_term = deform.point_cell_integral(np.array(0.0), np.array(0.0), hx, hx)
    assert abs(float(self_term) - 4 * hx * np.arcsinh(1.0)) < 1e-14


def test_point_direct_sum_vs_quadruple_loop():
    rng = np.random.default_rng(0)
    Nx, Ny, hx, hy = 7, 5, 0.3, 0.2
    P = rng.random((Nx, Ny))
    k2 = deform.point_kernel(Nx, Ny, hx, hy)
    H = np.zeros((Nx, Ny))
    for i in range(Nx):
        for j in range(Ny):
            s = 0.0
            for a in range(Nx):
                for b in range(Ny):
                    s += k2[abs(i - a), abs(j - b)] * P[a, b]
            H[i, j] = s
    assert np.abs(deform.point_deformation(P, hx, hy) - H).max() < 1e-13


def test_point_hertz_identity():
    errs = []
    for n in [33, 65]:
        x = np.linspace(-1.5, 1.5, n)
        h = x[1] - x[0]
        X, Y = np.meshgrid(x, x, indexing="ij")
        P = np.sqrt(np.clip(1 - X * X - Y * Y, 0, None))
        H = 0.5 * (X * X + Y * Y) + deform.point_deformation(P, h, h)
        inside = X * X + Y * Y < 0.5
        errs.append(np.abs(H[inside] - 1.0).max())
    assert errs[1] < errs[0] < 0.05


def _fd_sigma_jacobian(P, H, ph, lam, h, D, T, kappa=None):
    """Central differences of sigma -> R(P + D sigma, H + T sigma)."""
    n = len(P) - 2
    J = np.zeros((n, n))
    e = 1e-7
    for k in range(n):
        s = np.zeros(n)
        s[k] = e
        Pp = P.copy(); Pp[1:-1] += D @ s
        Pm = P.copy(); Pm[1:-1] -= D @ s
        Rp, _ = E.residual(Pp, H + T @ np.concatenate([[0], s, [0]]), ph, lam, h, kappa)
        Rm, _ = E.residual(Pm, H - T @ np.concatenate([[0], s, [0]]), ph, lam, h, kappa)
        J[:, k] = (Rp - Rm) / (2 * e)
    return J


@pytest.mark.parametrize("kterms,kappa", [(1, None), (2, None), (2, 0.0), (2, 1.0 / 3.0),
                                          (1, -1.0)])
def test_band_jacobian_matches_finite_differences(kterms, kappa):
    N = 65
    M, L = 20.0, 10.0
    x, h = E.grid(N)
    kvec = deform.line_kernel(N, h)
    _, lam, ph = E.moes_line(M, L)
    rng = np.random.default_rng(3)
    P = E.hertz_start(x) * (1 + 0.1 * rng.random(N))
    P[0] = P[-1] = 0.0
    P[45:50] = 0.0  # a cavitated patch
    H = E.film(P, -0.3, x, kvec)
    direct = rng.random(N - 2) < 0.5
    n = N - 2
    # D and the truncated distributed kernel T = (K D) cut to |m - k| <= kterms
    D = np.eye(n)
    for k in range(n):
        if not direct[k]:
            if k > 0:
                D[k - 1, k] = -0.5
            if k < n - 1:
                D[k + 1, k] = -0.5
    K = deform.line_matrix(N, h)
    Dfull = np.zeros((N, N))
    Dfull[1:-1, 1:-1] = D
    KD = K @ Dfull
    T = np.zeros((N, N))
    for m in range(N):
        for k in range(1, N - 1):
            if abs(m - k) <= kterms:
                T[m, k] = KD[m, k]
    Jfd = _fd_sigma_jacobian(P, H, ph, lam, h, D, T, kappa)
    J = E.jacobian_band(P, H, ph, lam, h, kvec, direct, kterms, limjac=0, kappa=kappa)
    Jd = np.zeros((n, n))
    for r in range(n):
        for s in range(-4, 5):
            if 0 <= r + s < n:
                Jd[r, r + s] = J[r, s + 4]
    assert np.abs(Jd - Jfd).max() <= 1e-6 * np.abs(Jfd).max()
    assert np.abs(np.triu(Jfd, 5)).max() == 0 and np.abs(np.tril(Jfd, -5)).max() == 0


@pytest.fixture(scope="module")
def converged_cfg1():
    r = E.solve_line(20.0, 10.0, 257)
    assert r["status"] == 0
    return r


def test_line_fixed_point_complementarity(converged_cfg1):
    r = converged_cfg1
    comp, load_err, Lop, H = E.complementarity(r["P"], r["H0"], r["x"], r["h"], r["kvec"], 20.0,
                                               10.0)
    P = r["P"]
    assert P.min() >= 0.0
    assert abs(load_err) < 1e-12
    scale = np.abs(Lop).max()
    assert Lop[P[1:-1] == 0].min() >= -1e-10 * scale
    assert comp < 1e-10 * scale
    assert H.min() > 0


def test_line_flux_invariant(converged_cfg1):
    """Where R_i = 0 on a run of pressurised nodes the face fluxes
    q_{i+1/2} = (rho H)*_{i+1/2} - eps_{i+1/2}(P_{i+1} - P_i)/h are equal."""
    r = converged_cfg1
    P, H, h = r["P"], r["H"], r["h"]
    _, lam, ph = E.moes_line(20.0, 10.0)
    st = E.state(P, H, ph, lam)
    eps, rH = st["eps"], st["rH"]
    epsh = 0.5 * (eps[:-1] + eps[1:])
    psi, _, _ = E.vanleer(rH[1:-1] - rH[:-2], rH[2:] - rH[1:-1])
    f = np.empty(len(P) - 1)
    f[0] = rH[0]
    f[1:] = rH[1:-1] + 0.5 * psi
    q = f - epsh * (P[1:] - P[:-1]) / h
    pos = np.where(P > 0)[0]
    # faces between the first and last pressurised node
    lo, hi = pos[0], pos[-1]
    qq = q[lo - 1:hi + 1]
    assert (qq.max() - qq.min()) < 1e-9 * np.abs(qq).max()


def test_line_solution_reference_values(converged_cfg1):
    """Context values of the converged config-1 solution (M=20, L=10, N=257):
    central film thickness of order 0.1 and a pressure close to Hertzian
    inside the contact (Moes M=20 is a moderately loaded contact)."""
    r = converged_cfg1
    x, P = r["x"], r["P"]
    assert 0.05 < r["Hmin"] < 0.1
    herz = E.hertz_start(x)
    assert np.abs(P - herz)[np.abs(x) < 0.5].max() < 0.1


def test_newton_stops_when_the_lcp_keeps_hitting_its_cap(monkeypatch):
    """The line iteration gives up with status 3 once the linearised LCP has
    hit its active-set cap in LCP_FAIL_STEPS consecutive steps (the GPU
    driver applies the same rule); an LCP that converges resets the count."""
    real = E.lcp_exact
    calls = {"n": 0}

    def capped(A, b, bnd, max_iter=64):
        calls["n"] += 1
        u, _ = real(A, b, bnd, max_iter)
        # one converged step in the middle resets the consecutive count
        return u, (0 if calls["n"] == 5 else E.LCP_NOT_CONVERGED)

    monkeypatch.setattr(E, "lcp_exact", capped)
    r = E.solve_line(20.0, 10.0, 65, max_newton=200)
    assert r["status"] == E.LCP_NOT_CONVERGED
    assert r["iters"] == 5 + E.LCP_FAIL_STEPS


def test_newton_stops_when_the_change_stalls(monkeypatch):
    """Status 6 before max_newton once max |P change| has set no new minimum
    for stall_steps steps (the GPU driver applies the same rule): a change
    that halves for 10 steps and then hovers above that minimum stops at step
    10 + stall_steps; with the rule off it runs to max_newton."""
    calls = {"n": 0}

    def fake_step(P, H0, *args):
        calls["n"] += 1
        k = calls["n"]
        size = 0.5 ** k if k <= 10 else 0.5 ** 10 * (1.5 if k % 2 else 1.2)
        Pn = P.copy()
        Pn[len(P) // 2] += size if k % 2 else -size
        return Pn, H0, {}

    monkeypatch.setattr(E, "newton_step", fake_step)
    r = E.solve_line(20.0, 10.0, 65, max_newton=2000, stall_steps=300)
    assert r["status"] == 6
    assert r["iters"] == 10 + 300
    calls["n"] = 0
    r = E.solve_line(20.0, 10.0, 65, max_newton=500)
    assert r["status"] == 6 and r["iters"] == 500


@pytest.mark.parametrize("kappa", [0.0, 1.0 / 3.0, -1.0, 0.5])
def test_kappa_slope_closed_form_on_a_cubic(kappa):
    """The kappa-scheme face values (rH)_{i+1/2} = (rH)_i + psi/2 of Sec. 3.3
    on rH = x^3: the flux difference is 3 x^2 + h^2 (3 kappa - 1)/2 exactly
    (third order only for kappa = 1/3); swapping the (1+kappa), (1-kappa)
    weights or halving psi fails it."""
    h = 0.01
    x = h * np.arange(-20, 21)
    rH = x ** 3
    psi, _, _ = E.slope(rH[1:-1] - rH[:-2], rH[2:] - rH[1:-1], kappa)
    f = rH[1:-1] + 0.5 * psi                   # faces i+1/2 for nodes 1..n-2
    diff = (f[1:] - f[:-1]) / h                # at nodes 2..n-2
    ref = 3 * x[2:-1] ** 2 + h * h * (3 * kappa - 1) / 2
    assert np.abs(diff - ref).max() <= 1e-10


@pytest.mark.parametrize("kappa", [0.0, 1.0 / 3.0, -1.0])
def test_converged_config1_with_kappa_scheme(kappa):
    """Config 1 with the kappa-scheme convection: complementarity, load
    balance, and the face-flux invariant on the pressurised run."""
    r = E.solve_line(20.0, 10.0, 257, tol=1e-13, max_newton=2000, kappa=kappa)
    assert r["status"] == 0
    P, H, h = r["P"], r["H"], r["h"]
    comp, load_err, Lop, _ = E.complementarity(P, r["H0"], r["x"], h, r["kvec"], 20.0, 10.0,
                                                kappa=kappa)
    scale = np.abs(Lop).max()
    assert abs(load_err) < 1e-12 and comp < 1e-10 * scale
    assert Lop[P[1:-1] == 0].min() >= -1e-10 * scale
    _, lam, ph = E.moes_line(20.0, 10.0)
    st = E.state(P, H, ph, lam)
    eps, rH = st["eps"], st["rH"]
    psi, _, _ = E.slope(rH[1:-1] - rH[:-2], rH[2:] - rH[1:-1], kappa)
    f = np.empty(len(P) - 1)
    f[0] = rH[0]
    f[1:] = rH[1:-1] + 0.5 * psi
    q = f - 0.5 * (eps[:-1] + eps[1:]) * (P[1:] - P[:-1]) / h
    pos = np.where(P > 0)[0]
    qq = q[pos[0] - 1:pos[-1] + 1]
    assert (qq.max() - qq.min()) < 1e-9 * np.abs(qq).max()


def _implicit_operator_line(sigma, P, H, eps, rho, h, D, T, c):
    """Implicit part of the splittings Lhs1 / Lhs2 as a function of the
    change sigma (interior nodes), written from eqs. 62 and 70 (1D): eps and
    rho stay at the current iterate, the pressure moves by D sigma, the film
    by T sigma (the distributed kernel cut as in eqs. 67 and 74), and the
    convective flux is the upwind value rho H of the node behind the face,
    weighted by c."""
    s = np.concatenate([[0.0], sigma, [0.0]])
    Pb = P.copy()
    Pb[1:-1] += D @ sigma
    Hb = H + T @ s
    ef = 0.5 * (eps[:-1] + eps[1:])
    dP = Pb[1:] - Pb[:-1]
    diff = (ef[1:] * dP[1:] - ef[:-1] * dP[:-1]) / h ** 2
    f = rho * Hb                                  # upwind face value of face i+1/2: node i
    return diff - c * (f[1:-1] - f[:-2]) / h


@pytest.mark.parametrize("split,kappa", [(1, None), (2, None), (1, 1.0 / 3.0), (2, 1.0 / 3.0),
                                         (2, -1.0)])
def test_splitting_band_matches_finite_differences(split, kappa):
    """The Lhs1 / Lhs2 matrix is the derivative of its implicit operator
    (finite differences of the function above, with distributive columns and
    the elastic film cut to |m - k| <= 2); the weights are (2 - k)/2 and
    (2 - k)/2 + (1 - k)/4 (k = 0 for the limited slope)."""
    N, kterms = 65, 2
    x, h = E.grid(N)
    kvec = deform.line_kernel(N, h)
    _, lam, ph = E.moes_line(50.0, 8.0)
    rng = np.random.default_rng(11)
    P = E.hertz_start(x) * (1 + 0.1 * rng.random(N))
    P[0] = P[-1] = 0.0
    P[40:44] = 0.0
    H = E.film(P, -0.2, x, kvec)
    st = E.state(P, H, ph, lam)
    n = N - 2
    direct = rng.random(n) < 0.5
    D = np.eye(n)
    for k in range(n):
        if not direct[k]:
            if k > 0:
                D[k - 1, k] = -0.5
            if k < n - 1:
                D[k + 1, k] = -0.5
    Dfull = np.zeros((N, N))
    Dfull[1:-1, 1:-1] = D
    KD = deform.line_matrix(N, h) @ Dfull
    T = np.zeros((N, N))
    for m in range(N):
        for k in range(1, N - 1):
            if abs(m - k) <= kterms:
                T[m, k] = KD[m, k]
    kk = 0.0 if kappa is None else kappa
    c = (2 - kk) / 2 if split == 1 else (2 - kk) / 2 + (1 - kk) / 4
    e = 1e-6
    Jfd = np.zeros((n, n))
    for k in range(n):
        s = np.zeros(n)
        s[k] = e
        Jfd[:, k] = (_implicit_operator_line(s, P, H, st["eps"], st["rho"], h, D, T, c) -
                     _implicit_operator_line(-s, P, H, st["eps"], st["rho"], h, D, T, c)) / (2 * e)
    J = E.jacobian_band(P, H, ph, lam, h, kvec, direct, kterms, kappa=kappa, split=split)
    Jd = np.zeros((n, n))
    for r in range(n):
        for s in range(-4, 5):
            if 0 <= r + s < n:
                Jd[r, r + s] = J[r, s + 4]
    err = np.abs(Jd - Jfd).max()
    assert err <= 1e-12 * np.abs(Jfd).max()
    # the test tells the matrices apart: the Newton band (eps, rho and the
    # slope move there) and the other splitting's weight differ by far more
    Jn = E.jacobian_band(P, H, ph, lam, h, kvec, direct, kterms, limjac=0, kappa=kappa)
    Jo = E.jacobian_band(P, H, ph, lam, h, kvec, direct, kterms, kappa=kappa, split=3 - split)
    assert np.abs(Jn - J).max() > 1e6 * err and np.abs(Jo - J).max() > 1e6 * err


@pytest.mark.parametrize("split", [1, 2])
def test_splitting_reaches_the_newton_fixed_point(split, converged_cfg1):
    """Lhs1 and Lhs2 change the iteration, not the discrete equations: on
    config 1 they converge to the Newton iteration's fixed point."""
    r = E.solve_line(20.0, 10.0, 257, splitting=split, max_newton=2000)
    assert r["status"] == 0
    ref = converged_cfg1
    assert np.abs(r["P"] - ref["P"]).max() <= 1e-10 * np.abs(ref["P"]).max()
    assert abs(r["H0"] - ref["H0"]) <= 1e-10 * abs(ref["H0"])
    assert abs(r["Hmin"] - ref["Hmin"]) <= 1e-10 * abs(ref["Hmin"])
