"""Oracle (test infrastructure): EHL line contact, FP64, following Sec. 3.3.

Problem (Example "line contact", Sec. 3.3): find the pressure P(X) >= 0 and
the constant H0 such that the Reynolds operator
    L(P) = d(rho H)/dX - d/dX(eps dP/dX) >= 0,   P L(P) = 0,
with P = 0 at both ends of X in [-4.5, 1.5] and the load balance
integral of P = pi/2, where
    H   = H0 + X^2/2 - (1/pi) int ln|X - X'| P(X') dX'  (+ roughness R(X)),
    eps = rho H^3 / (eta lam),
    eta = exp{(alpha p0 / z)(-1 + (1 + p_h P / p0)^z)}         (Roelands),
    rho = (0.59e9 + 1.34 p_h P) / (0.59e9 + p_h P)             (Dowson-Higginson).

Moes parameters (appendix): L = G (2U)^(1/4), M = W (2U)^(-1/2); with the
Hertzian line-contact half width b = R sqrt(8W/pi) and p_h = E' sqrt(W/2pi)
these give alpha_bar = alpha p_h = L sqrt(M / (2 pi)) and
lam = 6 eta0 u_s R^2 / (b^3 p_h) = 3 pi^2 / (8 M^2).  alpha = 1.7e-8 1/Pa,
p0 = 1.98e8 Pa, z = 0.68.

Discretisation (Sec. 3.3.3, eqs. 62-65, in one dimension): nodes
X_i = -4.5 + i h, i = 0..N-1, h = 6/(N-1); unknowns P_1..P_{N-2};
    R_i = [eps_{i+1/2}(P_{i+1} - P_i) - eps_{i-1/2}(P_i - P_{i-1})] / h^2
          - [(rho H)*_{i+1/2} - (rho H)*_{i-1/2}] / h,
    eps_{i+-1/2} = (eps_i + eps_{i+-1}) / 2,
    (rho H)*_{i+1/2} = (rho H)_i + psi_i / 2,  psi_0 = 0,
    psi_i = (D+ |D-| + |D+| D-) / (|D+| + |D-|)   (van Leer limited slope,
            D- = (rho H)_i - (rho H)_{i-1}, D+ = (rho H)_{i+1} - (rho H)_i;
            psi = 0 when both vanish),
and L_i = -R_i.  Readings: the limiter function is not named in the paper
(van Leer, a symmetric limiter, is used); the printed ratio r = D+/D- with
phi(r) D+ is read as the Sweby form phi(D-/D+)... which for a symmetric
limiter equals psi above.  The flow is in +X.

Iteration (the paper's hybrid Newton line method Lhs1, eqs. 60, 62-68, 75):
  * band Jacobian J = dR/dP of the local terms, with the elastic kernel
    coupling dH_k/dP_j kept only for |k - j| <= kterms (eq. 67 keeps three
    terms, kterms = 1; the default here keeps five, kterms = 2, without which
    the iteration diverges from the Hertzian start on grids of 2049 nodes);
  * hybrid switch (eq. 60): node i takes a direct change (Ls1) when
    eps_i / h > 0.6, else a weighted (distributive) change (Ls4): the change
    vector is delta = D sigma where column i of D is e_i for a direct node
    and e_i - (e_{i-1} + e_{i+1})/2 for a distributive node (the 1D form of
    the quarter weights of eq. 69 -- a reading, the paper prints only 2D);
  * the linearised complementarity problem in v = P + sigma,
        A = -J D,  b = A P + R,   v >= 0, A v - b >= 0, v (A v - b) = 0,
    is posed on the rows whose node and both neighbours are direct; other
    rows are free; it is solved exactly (active set on the AQIF solve);
  * update P <- max(0, P + omega D (v - P)), then the load balance
    H0 <- H0 - c (pi/2 - h sum P)  (eq. 75, line form).
The fixed point (P >= 0, L >= 0, P L = 0, h sum P = pi/2) does not depend on
omega, c or the starting point; those are passed in explicitly.
"""
import numpy as np

from . import deform

ALPHA = 1.7e-8
P0_ROELANDS = 1.98e8
Z_ROELANDS = 0.68
RHO_A = 0.59e9
RHO_B = 1.34
XA, XB = -4.5, 1.5
SWITCH = 0.6
LIMJAC = 2   # limiter terms of the Newton matrix (see limiter_jacobian)
LCP_NOT_CONVERGED = 3   # status: the step's LCP hit its active-set cap ...
LCP_FAIL_STEPS = 16     # ... in this many consecutive Newton steps


def moes_line(M, L):
    """(alpha_bar, lam, p_h) of the line contact from the Moes M, L."""
    abar = L * np.sqrt(M / (2.0 * np.pi))
    lam = 3.0 * np.pi ** 2 / (8.0 * M ** 2)
    return abar, lam, abar / ALPHA


def grid(N, xa=XA, xb=XB):
    h = (xb - xa) / (N - 1)
    return xa + h * np.arange(N), h


def hertz_start(x):
    return np.sqrt(np.clip(1.0 - x * x, 0.0, None))


def lubricant(P, ph):
    """rho, d rho/dP, ln eta, d ln eta/dP (all node-wise)."""
    s = ph / P0_ROELANDS
    base = 1.0 + s * P
    c = ALPHA * P0_ROELANDS / Z_ROELANDS
    lneta = c * (-1.0 + base ** Z_ROELANDS)
    dlneta = c * Z_ROELANDS * base ** (Z_ROELANDS - 1.0) * s
    rho = (RHO_A + RHO_B * ph * P) / (RHO_A + ph * P)
    drho = (RHO_B * ph * (RHO_A + ph * P) - (RHO_A + RHO_B * ph * P) * ph) / (RHO_A + ph * P) ** 2
    return rho, drho, lneta, dlneta


def film(P, H0, x, kvec, rough=None):
    """H_i = H0 + X_i^2/2 + sum_j k[|i-j|] P_j (+ roughness)."""
    N = len(P)
    idx = np.abs(np.arange(N)[:, None] - np.arange(N)[None, :])
    H = H0 + 0.5 * x * x + kvec[idx] @ P
    if rough is not None:
        H = H + rough
    return H


def vanleer(dm, dp):
    """psi and its partial derivatives wrt D+ (dp) and D- (dm)."""
    same = dm * dp > 0.0
    den = np.where(same, dp + dm, 1.0)
    psi = np.where(same, 2.0 * dp * dm / den, 0.0)
    dpsi_dp = np.where(same, 2.0 * dm * dm / (den * den), 0.0)
    dpsi_dm = np.where(same, 2.0 * dp * dp / (den * den), 0.0)
    return psi, dpsi_dp, dpsi_dm


def slope(dm, dp, kappa=None):
    """Slope psi of the convective face value (rH)_{i+1/2} = (rH)_i + psi/2
    and its partials wrt D+ and D-: the van Leer limited slope (TVD, the
    method's default), or with kappa given the kappa-scheme of Sec. 3.3 (eqs.
    56-59), psi = (1+kappa)/2 D+ + (1-kappa)/2 D-, linear and unlimited."""
    if kappa is None:
        return vanleer(dm, dp)
    return (0.5 * (1.0 + kappa) * dp + 0.5 * (1.0 - kappa) * dm,
            np.full(np.shape(dp), 0.5 * (1.0 + kappa)), np.full(np.shape(dm), 0.5 * (1.0 - kappa)))


def limiter_jacobian(dm, dp, mode, kappa=None):
    """Limiter coefficients (pa = d/dD+, pb = d/dD-) used in the Newton
    matrix; the residual always uses psi.  mode 0: exact derivatives of psi;
    1: the ratio frozen at the current iterate, psi = phi(r) D- with r = D+/D-,
    phi(r) = 2r/(1+r) held fixed (eqs. 64-65 evaluate r from the old film), so
    pa = 0, pb = phi; 2: first-order upwind flux, pa = pb = 0.  For the
    kappa-scheme (linear) modes 0 and 1 are both its exact constants."""
    if kappa is not None:
        _, pa, pb = slope(dm, dp, kappa)
        if mode == 2:
            return np.zeros_like(pa), np.zeros_like(pb)
        return pa, pb
    _, pa, pb = vanleer(dm, dp)
    if mode == 0:
        return pa, pb
    same = dm * dp > 0.0
    phi = np.where(same, 2.0 * dp / np.where(same, dm + dp, 1.0), 0.0)
    if mode == 1:
        return np.zeros_like(pa), phi
    return np.zeros_like(pa), np.zeros_like(pb)


def splitting_coefficient(split, kappa=None):
    """Weight of the upwind film-response difference (rho H)_i - (rho H)_{i-1}
    in the implicit operator of the paper's hybrid splittings (Sec. 3.3.2):
    Lhs1 (eq. 60: Ls1 for a direct change, eq. 49; Ls4 for a weighted change,
    eqs. 56-57) keeps (2 - kappa)/2 of it implicit; Lhs2 (eq. 61: Ls0, eq. 48;
    Ls5, eqs. 58-59) also moves the (1 - kappa)/4 part of the upstream
    difference, (H_{i-1} - H_i) + (H_i - H_{i-2}), to the implicit side:
    (2 - kappa)/2 + (1 - kappa)/4.  kappa = 0 with the limited slope."""
    k = 0.0 if kappa is None else kappa
    if split == 1:
        return 0.5 * (2.0 - k)
    if split == 2:
        return 0.5 * (2.0 - k) + 0.25 * (1.0 - k)
    raise ValueError("split must be 1 (Lhs1) or 2 (Lhs2)")


def state(P, H, ph, lam):
    rho, drho, lneta, dlneta = lubricant(P, ph)
    eta = np.exp(lneta)
    eps = rho * H ** 3 / (eta * lam)
    return dict(rho=rho, drho=drho, dlneta=dlneta, eta=eta, eps=eps, rH=rho * H, H=H)


def residual(P, H, ph, lam, h, kappa=None):
    """R_i for interior i (array of length N-2), plus the state (convective
    slope: van Leer, or the kappa-scheme when kappa is given)."""
    s = state(P, H, ph, lam)
    eps, rH = s["eps"], s["rH"]
    epsh = 0.5 * (eps[:-1] + eps[1:])             # faces i+1/2, i = 0..N-2
    psi, _, _ = slope(rH[1:-1] - rH[:-2], rH[2:] - rH[1:-1], kappa)
    f = np.empty(len(P) - 1)
    f[0] = rH[0]
    f[1:] = rH[1:-1] + 0.5 * psi
    dP = P[1:] - P[:-1]
    R = (epsh[1:] * dP[1:] - epsh[:-1] * dP[:-1]) / h ** 2 - (f[1:] - f[:-1]) / h
    return R, s


def jacobian_band(P, H, ph, lam, h, kvec, direct=None, kterms=1, limjac=0, kappa=None,
                  split=0):
    """Band of dR_i/dsigma_j (interior rows and columns) for the change
    delta = D sigma (column j of D: e_j for a direct node, e_j - (e_{j-1} +
    e_{j+1})/2 for a distributive one; boundary nodes stay fixed).

    The film reacts to sigma_j through the distributed kernel (K D); as in
    eqs. 66-67 and 74 it is kept for the nodes |m - j| <= kterms only.
    With every node direct this is dR/dP with the kernel cut to |k-j| <= 1.
    split = 1 or 2: the implicit operator of the splitting Lhs1 or Lhs2
    instead -- eps and rho held at the current iterate (eqs. 62, 64-65,
    70, 72-73: only P + D sigma and the film H + K D sigma move), the
    convective flux first-order upwind with the weight
    splitting_coefficient(split, kappa).
    Returns J with J[r, s+4] = dR_{r+1}/dsigma_{r+1+s}, s = -4..4 (nonzero
    offsets -3..2)."""
    N = len(P)
    n = N - 2
    if direct is None:
        direct = np.ones(n, dtype=bool)
    dist = np.zeros(N, dtype=bool)
    dist[1:-1] = ~np.asarray(direct, dtype=bool)
    interior = np.zeros(N, dtype=bool)
    interior[1:-1] = True
    st = state(P, H, ph, lam)
    rho, drho, dlneta, eps, rH = st["rho"], st["drho"], st["dlneta"], st["eps"], st["rH"]
    lam_eta = st["eta"] * lam
    m = np.arange(N)

    def Dcol(k, jrow):
        """D[jrow, k] for arrays (k interior column, jrow node)."""
        out = np.where(jrow == k, 1.0, 0.0)
        nb = (np.abs(jrow - k) == 1) & dist[np.clip(k, 0, N - 1)] & interior[np.clip(jrow, 0, N - 1)]
        return np.where(nb, -0.5, out)

    def kap(d):
        d = np.abs(d)
        return np.where(d < N, kvec[np.clip(d, 0, N - 1)], 0.0)

    # node derivatives wrt sigma_{m+o}, |o| <= kterms (film) / 1 (pressure)
    OFFS = tuple(range(-kterms, kterms + 1))
    dPn, dHn = {}, {}
    for o in OFFS:
        k = m + o
        kin = (k >= 1) & (k <= N - 2)
        dPn[o] = np.where(kin & (abs(o) <= 1), Dcol(k, m), 0.0)
        # (K D)[m, k] = kappa(m-k) - (kappa(m-k+1) [k-1 interior] + kappa(m-k-1) [k+1 interior])/2
        kd = kap(m - k)
        dk = dist[np.clip(k, 0, N - 1)]
        corr = 0.5 * (np.where(interior[np.clip(k - 1, 0, N - 1)], kap(m - k + 1), 0.0) +
                      np.where(interior[np.clip(k + 1, 0, N - 1)], kap(m - k - 1), 0.0))
        dHn[o] = np.where(kin, np.where(dk, kd - corr, kd), 0.0)
    eP = drho * H ** 3 / lam_eta - eps * dlneta
    eH = 3.0 * rho * H ** 2 / lam_eta
    drhoH = drho * H
    cw = 1.0
    if split:
        eP, eH, drhoH = 0.0 * eP, 0.0 * eH, 0.0 * drhoH
        limjac, cw = 2, splitting_coefficient(split, kappa)
    deps = {o: eP * dPn[o] + eH * dHn[o] for o in OFFS}
    drH = {o: drhoH * dPn[o] + rho * dHn[o] for o in OFFS}

    def node_d(darr, mm, j):
        o = j - mm
        out = np.zeros(len(mm))
        for oo in OFFS:
            sel = (o == oo) & (mm >= 0) & (mm < N)
            out[sel] = darr[oo][mm[sel]]
        return out

    epsh = 0.5 * (eps[:-1] + eps[1:])
    dm = rH[1:-1] - rH[:-2]
    dp = rH[2:] - rH[1:-1]
    pa, pb = limiter_jacobian(dm, dp, limjac, kappa)  # index t -> node t+1
    i = np.arange(1, N - 1)
    J = np.zeros((n, 9))
    for s in range(-4, 5):
        j = i + s
        valid = (j >= 1) & (j <= N - 2)
        de_p = 0.5 * (node_d(deps, i, j) + node_d(deps, i + 1, j))
        de_m = 0.5 * (node_d(deps, i - 1, j) + node_d(deps, i, j))
        dPi, dPp, dPm = node_d(dPn, i, j), node_d(dPn, i + 1, j), node_d(dPn, i - 1, j)
        dA = de_p * (P[i + 1] - P[i]) + epsh[i] * (dPp - dPi)
        dB = de_m * (P[i] - P[i - 1]) + epsh[i - 1] * (dPi - dPm)

        def dflux(fi):
            # d f_{fi+1/2}/dsigma_j; f_0 = rH_0, f_t = rH_t + psi_t / 2
            out = node_d(drH, fi, j)
            t = fi >= 1
            ft = fi[t]
            dpsi = pa[ft - 1] * (node_d(drH, ft + 1, j[t]) - node_d(drH, ft, j[t])) + \
                pb[ft - 1] * (node_d(drH, ft, j[t]) - node_d(drH, ft - 1, j[t]))
            out[t] += 0.5 * dpsi
            return out

        dR = (dA - dB) / h ** 2 - cw * (dflux(i) - dflux(i - 1)) / h
        J[:, s + 4] = np.where(valid, dR, 0.0)
    return J


def distributive_matrix_band(direct):
    """D (interior columns): column i = e_i (direct) or e_i - (e_{i-1}+e_{i+1})/2.
    Returned as a band with D[r, o+1] = D[r, r+o], o in {-1, 0, 1}."""
    n = len(direct)
    D = np.zeros((n, 3))
    D[:, 1] = 1.0
    dist = ~direct
    # D[r, r+1] = -1/2 if column r+1 distributive; D[r, r-1] = -1/2 if column r-1 distributive
    D[:-1, 2] = np.where(dist[1:], -0.5, 0.0)
    D[1:, 0] = np.where(dist[:-1], -0.5, 0.0)
    return D


def band_times_band(J, D):
    """(J D) as a band of half-width 4 (J: half-width 4, D: half-width 1)."""
    n = J.shape[0]
    out = np.zeros((n, 9))
    for s in range(-4, 5):
        for o in (-1, 0, 1):
            # (J D)[r, c] = sum_m J[r, m] D[m, c], m = r + s, c = m + o
            t = s + o
            if abs(t) > 4:
                continue
            r = np.arange(n)
            m = r + s
            ok = (m >= 0) & (m < n) & (m + o >= 0) & (m + o < n)
            out[ok, t + 4] += J[ok, s + 4] * D[m[ok], o + 1]
    return out


def band_matvec(A, v):
    n = A.shape[0]
    q = (A.shape[1] - 1) // 2
    out = np.zeros(n)
    for s in range(-q, q + 1):
        r = np.arange(n)
        c = r + s
        ok = (c >= 0) & (c < n)
        out[ok] += A[ok, s + q] * v[c[ok]]
    return out


def hybrid_direct(P, eps, h):
    """Hybrid switch (eq. 60): direct change where eps/h > 0.6, weighted
    (distributive) change elsewhere.  Reading at the free boundary: a node
    with a cavitated neighbour (P = 0 at i-1, i or i+1) also takes the direct
    change, so that the complementarity of the linearised problem acts on the
    node that actually reaches P = 0 (the paper does not say how the weighted
    change meets the cavitation boundary)."""
    direct = eps / h > SWITCH
    cav = P <= 0.0
    near = cav.copy()
    near[1:] |= cav[:-1]
    near[:-1] |= cav[1:]
    return direct | near


def newton_step(P, H0, x, h, kvec, M, L, rough, omega, c_h0, lcp_solve, kterms=2, limjac=LIMJAC,
                kappa=None, split=0):
    """One step of the hybrid line iteration (kappa given: the kappa-scheme
    convection of Sec. 3.3 instead of the limited slope; split 1 / 2: the
    implicit operator of the splitting Lhs1 / Lhs2 instead of the Newton
    band); returns (P_new, H0_new, info)."""
    abar, lam, ph = moes_line(M, L)
    H = film(P, H0, x, kvec, rough)
    R, st = residual(P, H, ph, lam, h, kappa)
    direct_all = hybrid_direct(P, st["eps"], h)
    direct = direct_all[1:-1]
    D = distributive_matrix_band(direct)
    A = -jacobian_band(P, H, ph, lam, h, kvec, direct, kterms, limjac, kappa, split)
    Pi = P[1:-1]
    b = band_matvec(A, Pi) + R
    nb = np.concatenate([[True], direct, [True]])
    bounded = (direct & nb[:-2] & nb[2:]).astype(np.uint8)
    v = lcp_solve(A, b, bounded)
    sigma = v - Pi
    delta = band_matvec(D, sigma)
    Pn = P.copy()
    Pn[1:-1] = np.maximum(0.0, Pi + omega * delta)
    load = h * Pn.sum()
    H0n = H0 - c_h0 * (np.pi / 2.0 - load)
    info = dict(R=R, delta=omega * delta, load=load, H=H, direct=direct_all, eps=st["eps"])
    return Pn, H0n, info


def complementarity(P, H0, x, h, kvec, M, L, rough=None, kappa=None):
    """max_i |min(P_i, L_i)| over interior nodes and the load error."""
    abar, lam, ph = moes_line(M, L)
    H = film(P, H0, x, kvec, rough)
    R, _ = residual(P, H, ph, lam, h, kappa)
    Lop = -R
    return np.abs(np.minimum(P[1:-1], Lop)).max(), np.pi / 2 - h * P.sum(), Lop, H


def start_h0(x, h, kvec, M):
    """Starting H0 (the paper is silent): with the Hertzian pressure, choose
    H0 so that the film in the Hertzian contact |X| <= 1 has its minimum at
    0.4 / sqrt(M):  H0 = 0.4/sqrt(M) - min_{|X_i| <= 1} (X_i^2/2 + H_el,i)."""
    P = hertz_start(x)
    P[0] = P[-1] = 0.0
    g = film(P, 0.0, x, kvec)
    return 0.4 / np.sqrt(M) - np.min(g[np.abs(x) <= 1.0])


def lcp_exact(A, b, bounded, max_iter=64):
    from . import lcp_solve, EXACT
    r = lcp_solve(A, b, bounded=bounded, mode=EXACT, max_iter=max_iter)
    return r["u"], r["status"]


def solve_line(M, L, N, omega=0.5, c_h0=0.1, kterms=2, max_newton=2000, tol=1e-13,
               rough=None, P=None, H0=None, limjac=None, stall_steps=0, kappa=None,
               rigid=False, lcp_max_iter=64, lcp_fail_steps=LCP_FAIL_STEPS, splitting=0):
    """Run the hybrid Newton line iteration to convergence.

    Stops when max |P_new - P| <= t * max(1, |P|_inf) and |pi/2 - h sum P|
    <= t, t = max(tol, 4 N eps) (status 0), when the linearised LCP hits its
    active-set cap (lcp_max_iter) in lcp_fail_steps consecutive steps
    (status 3), when
    max |P change| has set no new minimum for stall_steps steps (status 6;
    0 = never), else status 6 after max_newton steps.  Returns a dict
    with P (N nodes), H0, H, Hmin (min over all nodes, first index), the
    number of steps and the status.  ``rigid`` drops the elastic
    deformation (K = 0); with L = 0 (p_h = 0) the lubricant is
    incompressible and isoviscous (rho = eta = 1), the rigid-isoviscous
    problem the paper names for incompressible flow.  ``splitting`` 1 or 2
    iterates with the implicit operator of Lhs1 or Lhs2 (eqs. 60-61) instead
    of the Newton band: same fixed point, another iteration."""
    x, h = grid(N)
    kvec = np.zeros(N) if rigid else deform.line_kernel(N, h)
    if P is None:
        P = hertz_start(x)
        P[0] = P[-1] = 0.0
    if H0 is None:
        H0 = start_h0(x, h, kvec, M)
    status = 6
    last = [0]

    def lcp(A, b, bnd):
        u, st = lcp_exact(A, b, bnd, lcp_max_iter)
        last[0] = st
        return u

    # the FP64 rounding floor of the change grows with N: stop at
    # max(tol, 4 N eps), eps = 2^-52
    tl = max(tol, 4.0 * N * np.finfo(np.float64).eps)
    it = 0
    fails = 0  # consecutive steps whose LCP hit the active-set cap
    best, best_it = np.inf, 0
    for it in range(1, max_newton + 1):
        Pn, H0, info = newton_step(P, H0, x, h, kvec, M, L, rough, omega, c_h0, lcp, kterms,
                                   LIMJAC if limjac is None else limjac, kappa, splitting)
        dP = np.abs(Pn - P).max()
        P = Pn
        fails = fails + 1 if last[0] == LCP_NOT_CONVERGED else 0
        if not np.isfinite(dP):
            status = 2
            break
        if dP <= tl * max(1.0, np.abs(P).max()) and abs(np.pi / 2 - h * P.sum()) <= tl:
            status = 0
            break
        if fails >= lcp_fail_steps:
            # the active-set iteration cycles: this linearisation has no
            # solution the iteration reaches, the Newton iteration is lost
            status = LCP_NOT_CONVERGED
            break
        if dP < best:
            best, best_it = dP, it
        elif stall_steps > 0 and it - best_it >= stall_steps:
            break  # stalled (limit cycle or drift above the rounding floor): status 6
    H = film(P, H0, x, kvec, rough)
    if status == 0 and H.min() <= 0.0:
        status = 5
    return dict(P=P, H0=H0, H=H, Hmin=H.min(), argmin=int(np.argmin(H)), iters=it,
                status=status, x=x, h=h, kvec=kvec)
