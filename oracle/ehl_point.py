"""Oracle (test infrastructure): EHL point contact, FP64, following Sec. 3.3.

Problem (Example 5): find P(X, Y) >= 0 and H0 with
    L(P) = d(rho H)/dX - div(eps grad P) >= 0,  P L(P) = 0,
P = 0 on the boundary of [x0, x1] x [y0, y1], and the load balance
hx hy sum P = 2 pi / 3, where
    H = H0 + X^2/2 + Y^2/2 + (2/pi^2) int int P / |r - r'|  (deform.point_*),
    eps = rho H^3 / (eta lam)  with the lubricant models of ehl_line.
Point-contact Moes map (the paper prints only the line-contact M formula):
with a^3 = 3 F R / (2 E'), p_h = 3 F / (2 pi a^2) and M = W (2U)^(-3/4),
    alpha_bar = alpha p_h = (L / pi) (3 M / 2)^(1/3),
    lam = 6 eta0 u_s R^2 / (a^3 p_h) = (128 pi^3 / (3 M^4))^(1/3).

Discretisation (eqs. 62-65 on the 2D grid, flow in +X): for interior (i, j)
    R_ij = [eps_{i+1/2,j}(P_{i+1,j}-P_ij) - eps_{i-1/2,j}(P_ij-P_{i-1,j})] / hx^2
         + [eps_{i,j+1/2}(P_{i,j+1}-P_ij) - eps_{i,j-1/2}(P_ij-P_{i,j-1})] / hy^2
         - [(rho H)*_{i+1/2,j} - (rho H)*_{i-1/2,j}] / hx,
face values eps_{i+-1/2,j} = (eps_ij + eps_{i+-1,j}) / 2 (eq. 63) and the TVD
flux of each x-row exactly as in the line contact (van Leer, psi = 0 at the
inlet face; optionally the kappa-scheme slope of Sec. 3.3, eqs. 56-59, as in
ehl_line.slope).

Iteration (alternating line sweeps, eqs. 60, 62, 66-75): one step is an
x-sweep followed by a y-sweep.  A sweep solves, for every interior line of
its direction at once, a banded complementarity problem (half-bandwidth 4)
in the line's own change sigma:
  * node classification (eq. 60): direct where min(eps/hx, eps/hy) > 0.6 or
    where the node or one of its four neighbours is cavitated, else
    weighted (distributive) change;
  * change pattern (eq. 69): a distributive node's sigma changes its own
    pressure by sigma and each interior neighbour (along and across the line)
    by -sigma/4; a direct node's only its own;
  * Jacobian of the line: along-line diffusion and (x-lines) the TVD flux as
    in the line contact; the film responds through the distributed kernel
    (eq. 74, with the 1/4 weights of eq. 69) cut to |k - i| <= kterms; the
    across-line diffusion through the node's own eps and the -sigma/4 moved
    to the neighbours across the line (eq. 70); for y-lines the x-flux of
    each row through rho H at the x-columns l-2 .. l+1 (kernel response at
    x-offsets -2..1 and the moved -sigma/4).  The eps changes of the
    neighbours across the line are left out (the Jacobian only steers the
    iteration; the fixed point is that of R);
  * LCP in v = P + sigma on rows whose node and both along-line neighbours
    are direct (others free), A = -J, b = A P + R;
  * y-lines act on the direct nodes only (a weighted-change node keeps its
    pressure: row v = P): in the Hertzian zone a y-line reaches the x-flux
    only through the x-difference of the film response, which gives no
    usable line matrix (the y-sweep diverges there); x-lines carry them;
  * lines are solved in two colours (odd line index, then even, the film
    re-evaluated in between): with all lines at once, weighted changes of
    neighbouring lines can cancel (sigma != 0, zero net change: false fixed
    points), and the x-flux ties each y-line to its upstream neighbours;
  * after all lines: P <- max(0, P + omega delta) with delta_ij = sigma_ij -
    (sum of sigma/4 from the distributive interior neighbours), "changes at
    the end of the sweep" (eq. 69), then H0 <- H0 - c (2 pi/3 - hx hy sum P)
    (eq. 75).
"""
import numpy as np

from . import deform
from . import ehl_line as EL

XA, XB, YA, YB = -4.5, 1.5, -3.0, 3.0
LOAD = 2.0 * np.pi / 3.0


def moes_point(M, L):
    """(alpha_bar, lam, p_h) of the point contact from the Moes M, L."""
    abar = (L / np.pi) * (1.5 * M) ** (1.0 / 3.0)
    lam = (128.0 * np.pi ** 3 / (3.0 * M ** 4)) ** (1.0 / 3.0)
    return abar, lam, abar / EL.ALPHA


def grid(Nx, Ny, xa=XA, xb=XB, ya=YA, yb=YB):
    hx = (xb - xa) / (Nx - 1)
    hy = (yb - ya) / (Ny - 1)
    return xa + hx * np.arange(Nx), ya + hy * np.arange(Ny), hx, hy


def hertz_start(X, Y):
    P = np.sqrt(np.clip(1.0 - X[:, None] ** 2 - Y[None, :] ** 2, 0.0, None))
    P[0, :] = P[-1, :] = P[:, 0] = P[:, -1] = 0.0
    return P


def film(P, H0, X, Y, hx, hy, rough=None):
    H = H0 + 0.5 * X[:, None] ** 2 + 0.5 * Y[None, :] ** 2 + deform.point_deformation(P, hx, hy)
    return H if rough is None else H + rough


def x_flux(rH, kappa=None):
    """(rho H)* at the faces i+1/2 of every x-row, f[t, :] for t = 0..Nx-2,
    and the slope derivatives pa = dpsi/dD+, pb = dpsi/dD- at nodes 1..Nx-2
    (van Leer; with kappa given the kappa-scheme slope of Sec. 3.3, eqs. 56-59)."""
    psi, pa, pb = EL.slope(rH[1:-1] - rH[:-2], rH[2:] - rH[1:-1], kappa)
    f = np.empty((rH.shape[0] - 1, rH.shape[1]))
    f[0] = rH[0]
    f[1:] = rH[1:-1] + 0.5 * psi
    return f, pa, pb


def residual(P, H, ph, lam, hx, hy, kappa=None):
    """R_ij on the interior nodes, shape (Nx-2, Ny-2), plus the state."""
    s = EL.state(P, H, ph, lam)
    eps, rH = s["eps"], s["rH"]
    ex = 0.5 * (eps[:-1, :] + eps[1:, :])        # faces i+1/2
    ey = 0.5 * (eps[:, :-1] + eps[:, 1:])        # faces j+1/2
    dPx = P[1:, :] - P[:-1, :]
    dPy = P[:, 1:] - P[:, :-1]
    f, _, _ = x_flux(rH, kappa)
    Rx = (ex[1:, 1:-1] * dPx[1:, 1:-1] - ex[:-1, 1:-1] * dPx[:-1, 1:-1]) / hx ** 2
    Ry = (ey[1:-1, 1:] * dPy[1:-1, 1:] - ey[1:-1, :-1] * dPy[1:-1, :-1]) / hy ** 2
    Rc = (f[1:, 1:-1] - f[:-1, 1:-1]) / hx
    return Rx + Ry - Rc, s


def classify(P, eps, hx, hy):
    """direct (True) / distributive node flags on the whole grid (eq. 60 plus
    the cavitation rule); boundary nodes are direct."""
    direct = np.minimum(eps / hx, eps / hy) > EL.SWITCH
    cav = P <= 0.0
    near = cav.copy()
    near[1:, :] |= cav[:-1, :]
    near[:-1, :] |= cav[1:, :]
    near[:, 1:] |= cav[:, :-1]
    near[:, :-1] |= cav[:, 1:]
    d = direct | near
    d[0, :] = d[-1, :] = d[:, 0] = d[:, -1] = True
    return d


def sweep_systems(P, H, st, ph, lam, hx, hy, k2, direct, axis, kterms=1, limjac=EL.LIMJAC,
                  kappa=None, split=0):
    """Band systems of every interior line of one sweep direction.

    axis = 0: x-lines (one per interior j, positions i); axis = 1: y-lines.
    split = 1 or 2: the implicit operator of the splitting Lhs1 or Lhs2
    (eps and rho held at the current iterate, first-order upwind convective
    derivative weighted by ehl_line.splitting_coefficient) instead of the
    Newton band.
    Returns (A, b, bounded) with A of shape (lines, n, 9), A[l, r, s+4] =
    -dR/dsigma between rows r and r+s of line l (n = interior positions)."""
    # generic layout G[line, pos]: along-line = axis 1, across-line = axis 0
    T = (lambda a: a.T) if axis == 0 else (lambda a: a)
    h_a, h_p = (hx, hy) if axis == 0 else (hy, hx)
    Pg, Hg = T(P), T(H)
    eps, rH, rho, drho = T(st["eps"]), T(st["rH"]), T(st["rho"]), T(st["drho"])
    lam_eta = T(st["eta"]) * lam
    eP = drho * Hg ** 3 / lam_eta - eps * T(st["dlneta"])
    eH = 3.0 * rho * Hg ** 2 / lam_eta
    drhoH = drho * Hg
    cw = 1.0
    if split:
        eP, eH, drhoH = 0.0 * eP, 0.0 * eH, 0.0 * drhoH
        limjac, cw = 2, EL.splitting_coefficient(split, kappa)
    dist = ~T(direct)
    nl, nn = Pg.shape                       # lines incl. boundary lines, nodes per line
    n = nn - 2
    # kernel along the line (G) and one line across (Gp)
    G = k2[:, 0] if axis == 0 else k2[0, :]
    Gp = k2[:, 1] if axis == 0 else k2[1, :]

    def kv(arr, d):
        d = np.abs(d)
        return np.where(d < len(arr), arr[np.clip(d, 0, len(arr) - 1)], 0.0)

    lines = np.arange(1, nl - 1)
    L_ = len(lines)
    pos = np.arange(nn)
    interior_pos = (pos >= 1) & (pos <= nn - 2)
    # node derivatives wrt sigma_k, k = m + o: dP[o][l, m], dH[o][l, m]
    OFFS = tuple(range(-max(1, kterms), max(1, kterms) + 1))
    dPn, dHn = {}, {}
    across_in = np.ones(L_, dtype=bool)           # both across-neighbour lines are
    up_in = (lines + 1) <= nl - 2                 # interior lines?
    dn_in = (lines - 1) >= 1
    for o in OFFS:
        k = pos + o
        kin = (k >= 1) & (k <= nn - 2)
        kc = np.clip(k, 0, nn - 1)
        dk = dist[lines][:, kc]                   # (L_, nn): is column k distributive
        # pressure: D[m, k]
        dp = np.where(o == 0, 1.0, 0.0) * np.ones((L_, nn))
        if abs(o) == 1:
            dp = np.where(dk & interior_pos[None, :], -0.25, 0.0)
        dPn[o] = np.where(kin[None, :] & (abs(o) <= 1), dp, 0.0)
        # film: (K D)[m, k] cut to |m - k| <= kterms
        kd = kv(G, -o) * np.ones((L_, nn))
        corr = 0.25 * (np.where(interior_pos[np.clip(k - 1, 0, nn - 1)], kv(G, -o + 1), 0.0) +
                       np.where(interior_pos[np.clip(k + 1, 0, nn - 1)], kv(G, -o - 1), 0.0))
        corr = corr[None, :] + 0.25 * kv(Gp, -o) * (up_in.astype(float) + dn_in.astype(float))[:, None]
        dHn[o] = np.where(kin[None, :] & (abs(o) <= kterms), np.where(dk, kd - corr, kd), 0.0)
    del across_in

    eps_l, P_l = eps[lines], Pg[lines]
    deps = {o: eP[lines] * dPn[o] + eH[lines] * dHn[o] for o in OFFS}
    drH = {o: drhoH[lines] * dPn[o] + rho[lines] * dHn[o] for o in OFFS}

    def nd(darr, m, j):
        """derivative of node quantity at positions m wrt sigma at positions j
        (arrays over rows), per line."""
        o = j - m
        out = np.zeros((L_, len(m)))
        for oo in OFFS:
            sel = (o == oo) & (m >= 0) & (m < nn)
            out[:, sel] = darr[oo][:, m[sel]]
        return out

    i = np.arange(1, nn - 1)
    eph = 0.5 * (eps_l[:, 1:-1] + eps_l[:, 2:])
    epm = 0.5 * (eps_l[:, :-2] + eps_l[:, 1:-1])
    # across-line faces and pressures
    e_up = 0.5 * (eps_l[:, 1:-1] + eps[lines + 1][:, 1:-1])
    e_dn = 0.5 * (eps_l[:, 1:-1] + eps[lines - 1][:, 1:-1])
    P_up, P_dn, P_c = Pg[lines + 1][:, 1:-1], Pg[lines - 1][:, 1:-1], P_l[:, 1:-1]
    dist_c = dist[lines][:, 1:-1]
    if axis == 0:
        pa, pb = EL.limiter_jacobian(rH[lines][:, 1:-1] - rH[lines][:, :-2],
                                     rH[lines][:, 2:] - rH[lines][:, 1:-1], limjac,
                                     kappa)  # node t at [:, t-1]
    else:
        # the x-flux of row j depends on rho H at x-columns l-2 .. l+1; their
        # response to sigma on column l: the -sigma/4 moved to the columns
        # l +- 1 and the distributed kernel at x-offset a
        pa_all, pb_all = EL.limiter_jacobian(rH[1:-1] - rH[:-2], rH[2:] - rH[1:-1],
                                             limjac, kappa)  # row t-1 -> column t

        def kx(a, d):
            return kv(k2[abs(a)], d)

        drH_a = {}
        for a in (-2, -1, 1):
            col = np.clip(lines + a, 0, nl - 1)
            col_int = ((lines + a) >= 1) & ((lines + a) <= nl - 2)
            dPa, dHa = {}, {}
            for o in OFFS:
                k = pos + o
                kin = (k >= 1) & (k <= nn - 2)
                kc = np.clip(k, 0, nn - 1)
                dk = dist[lines][:, kc]
                mv = np.where(dk & (o == 0) & interior_pos[None, :] & col_int[:, None]
                              & (abs(a) == 1), -0.25, 0.0)
                dPa[o] = np.where(kin[None, :], mv, 0.0)
                kd = kx(a, -o) * np.ones((L_, nn))
                corr = 0.25 * (np.where(interior_pos[np.clip(k - 1, 0, nn - 1)], kx(a, -o + 1), 0.0) +
                               np.where(interior_pos[np.clip(k + 1, 0, nn - 1)], kx(a, -o - 1), 0.0))
                corr = corr[None, :] + 0.25 * (kx(a - 1, -o) * up_in.astype(float) +
                                               kx(a + 1, -o) * dn_in.astype(float))[:, None]
                dHa[o] = np.where(kin[None, :] & (abs(o) <= kterms),
                                  np.where(dk, kd - corr, kd), 0.0)
            drH_a[a] = {o: drhoH[col] * dPa[o] + rho[col] * dHa[o] for o in OFFS}
        drH_a[0] = drH
        pa_l, pb_l = pa_all[lines - 1], pb_all[lines - 1]
        pa_m = pa_all[np.clip(lines - 2, 0, None)]
        pb_m = pb_all[np.clip(lines - 2, 0, None)]
        first = (lines - 1 == 0)[:, None]
    J = np.zeros((L_, n, 9))
    for s in range(-4, 5):
        j = i + s
        valid = (j >= 1) & (j <= nn - 2)
        de_p = 0.5 * (nd(deps, i, j) + nd(deps, i + 1, j))
        de_m = 0.5 * (nd(deps, i - 1, j) + nd(deps, i, j))
        dPi, dPp, dPm = nd(dPn, i, j), nd(dPn, i + 1, j), nd(dPn, i - 1, j)
        dA = de_p * (P_l[:, 2:] - P_c) + eph * (dPp - dPi)
        dB = de_m * (P_c - P_l[:, :-2]) + epm * (dPi - dPm)
        along = (dA - dB) / h_a ** 2
        # across the line: own eps, own pressure and -sigma/4 moved across
        dEi = nd(deps, i, j)
        moved = np.where((s == 0) & dist_c, -0.25, 0.0)
        d_up = moved * up_in[:, None]
        d_dn = moved * dn_in[:, None]
        across = (0.5 * dEi * (P_up - P_c) + e_up * (d_up - dPi)
                  - 0.5 * dEi * (P_c - P_dn) - e_dn * (dPi - d_dn)) / h_p ** 2
        if axis == 0:
            def dflux(fi):
                out = nd(drH, fi, j)
                t = fi >= 1
                ft = fi[t]
                dpsi = pa[:, ft - 1] * (nd(drH, ft + 1, j[t]) - nd(drH, ft, j[t])) + \
                    pb[:, ft - 1] * (nd(drH, ft, j[t]) - nd(drH, ft - 1, j[t]))
                out[:, t] += 0.5 * dpsi
                return out
            conv = (dflux(i) - dflux(i - 1)) / h_a
        else:
            d = {a: nd(drH_a[a], i, j) for a in (-2, -1, 0, 1)}
            sl = slice(1, -1)
            f_i = (-0.5 * pb_l[:, sl] * d[-1] + (1.0 + 0.5 * (pb_l[:, sl] - pa_l[:, sl])) * d[0]
                   + 0.5 * pa_l[:, sl] * d[1])
            f_m = np.where(first, d[-1],
                           -0.5 * pb_m[:, sl] * d[-2]
                           + (1.0 + 0.5 * (pb_m[:, sl] - pa_m[:, sl])) * d[-1]
                           + 0.5 * pa_m[:, sl] * d[0])
            conv = (f_i - f_m) / h_p
        dR = along + across - cw * conv
        J[:, :, s + 4] = np.where(valid[None, :], dR, 0.0)
    A = -J
    R2, _ = residual(P, H, ph, lam, hx, hy, kappa)
    Rl = T(R2)                                   # (lines, n)
    b = np.einsum("lrs,lrs->lr", A, _shifted(P_l[:, 1:-1])) + Rl
    dr = T(direct)[lines]
    bounded = (dr[:, 1:-1] & dr[:, :-2] & dr[:, 2:]).astype(np.uint8)
    if axis == 1:
        # y-lines act on the direct nodes only: a weighted-change node keeps
        # its pressure (row v_r = P_r, free)
        frozen = ~dr[:, 1:-1]
        A[frozen] = 0.0
        A[frozen, 4] = 1.0
        b[frozen] = P_l[:, 1:-1][frozen]
        bounded[frozen] = 0
    return A, b, bounded


def _shifted(v):
    """v[l, r+s] arranged as (lines, n, 9) with zeros outside the line."""
    L_, n = v.shape
    out = np.zeros((L_, n, 9))
    for s in range(-4, 5):
        r = np.arange(n)
        c = r + s
        ok = (c >= 0) & (c < n)
        out[:, ok, s + 4] = v[:, c[ok]]
    return out


def sweep_update(P, sigma_g, direct, omega):
    """P <- max(0, P + omega delta), delta = sigma - sum of sigma/4 of the
    distributive interior neighbours (sigma_g on the whole grid, 0 on the
    boundary)."""
    dist = ~direct
    w = np.where(dist, sigma_g, 0.0)
    delta = sigma_g.copy()
    delta[1:, :] -= 0.25 * w[:-1, :]
    delta[:-1, :] -= 0.25 * w[1:, :]
    delta[:, 1:] -= 0.25 * w[:, :-1]
    delta[:, :-1] -= 0.25 * w[:, 1:]
    Pn = P.copy()
    Pn[1:-1, 1:-1] = np.maximum(0.0, P[1:-1, 1:-1] + omega * delta[1:-1, 1:-1])
    return Pn


def _sweep_part(P, H0, X, Y, hx, hy, k2, M, L, axis, omega, kterms, lcp, rough, color,
                kappa=None, split=0):
    """Solve the lines of one sweep direction (color None: all lines, else
    the lines whose index has that parity) and apply their changes."""
    _, lam, ph = moes_point(M, L)
    H = film(P, H0, X, Y, hx, hy, rough)
    st = EL.state(P, H, ph, lam)
    direct = classify(P, st["eps"], hx, hy)
    A, b, bounded = sweep_systems(P, H, st, ph, lam, hx, hy, k2, direct, axis, kterms,
                                  kappa=kappa, split=split)
    T = (lambda a: a.T) if axis == 0 else (lambda a: a)
    Pl = T(P)[1:-1, 1:-1]
    frozen = ~T(direct)[1:-1, 1:-1] if axis == 1 else np.zeros(Pl.shape, dtype=bool)
    sig = np.zeros_like(Pl)
    for l in range(A.shape[0]):
        if color is not None and (l + 1) % 2 != color:
            continue
        v = lcp(A[l], b[l], bounded[l])
        sig[l] = np.where(frozen[l], 0.0, v - Pl[l])
    sigma_g = np.zeros_like(P)
    sigma_g[1:-1, 1:-1] = sig.T if axis == 0 else sig
    return sweep_update(P, sigma_g, direct, omega)


def half_sweep(P, H0, X, Y, hx, hy, k2, M, L, axis, omega, c_h0, kterms, lcp, rough=None,
               kappa=None, split=0):
    """One sweep direction then the H0 update.  The lines are solved in two
    colours (odd lines, then even ones with the film re-evaluated): with all
    lines at once the weighted changes of neighbouring lines can cancel
    (sigma != 0 with zero net change, a false fixed point), and for y-lines
    the x-flux couples each column to its upstream neighbours."""
    for color in (1, 0):
        P = _sweep_part(P, H0, X, Y, hx, hy, k2, M, L, axis, omega, kterms, lcp, rough, color,
                        kappa, split)
    H0n = H0 - c_h0 * (LOAD - hx * hy * P.sum())
    return P, H0n


def start_h0(X, Y, hx, hy, M):
    """Starting H0 (the paper is silent): with the Hertzian pressure, the
    film inside the Hertzian circle has its minimum at 0.4 / M^(1/3)...
    scaled like the line-contact rule: H0 = 0.4 M^(-1/2) - min over the
    circle of (X^2 + Y^2)/2 + H_el."""
    P = hertz_start(X, Y)
    g = film(P, 0.0, X, Y, hx, hy)
    inside = X[:, None] ** 2 + Y[None, :] ** 2 <= 1.0
    return 0.4 / np.sqrt(M) - g[inside].min()


def solve_point(M, L, Nx, Ny, omega=0.5, c_h0=0.02, kterms=2, max_steps=400, tol=1e-12,
                rough=None, P=None, H0=None, lcp=None, kappa=None, splitting=0):
    """Alternating x/y line sweeps to convergence (splitting 1 / 2: the
    lines' matrices are the implicit operators of Lhs1 / Lhs2).  Stops when max |P change|
    over one x+y step <= t max(1, |P|_inf) and |2pi/3 - hx hy sum P| <= t,
    t = max(tol, 4 max(Nx, Ny) eps) (status 0), else status 6.  Returns dict(P, H0, H, Hmin, iters, status,
    X, Y, hx, hy)."""
    X, Y, hx, hy = grid(Nx, Ny)
    k2 = deform.point_kernel(Nx, Ny, hx, hy)
    if P is None:
        P = hertz_start(X, Y)
    if H0 is None:
        H0 = start_h0(X, Y, hx, hy, M)
    if lcp is None:
        lcp = lambda A, b, bd: EL.lcp_exact(A, b, bd)[0]
    status = 6
    tl = max(tol, 4.0 * max(Nx, Ny) * np.finfo(np.float64).eps)
    it = 0
    for it in range(1, max_steps + 1):
        P1, H0 = half_sweep(P, H0, X, Y, hx, hy, k2, M, L, 0, omega, c_h0, kterms, lcp, rough,
                            kappa, splitting)
        P2, H0 = half_sweep(P1, H0, X, Y, hx, hy, k2, M, L, 1, omega, c_h0, kterms, lcp, rough,
                            kappa, splitting)
        dP = np.abs(P2 - P).max()
        P = P2
        if not np.isfinite(dP):
            status = 2
            break
        if dP <= tl * max(1.0, np.abs(P).max()) and abs(LOAD - hx * hy * P.sum()) <= tl:
            status = 0
            break
    H = film(P, H0, X, Y, hx, hy, rough)
    if status == 0 and H.min() <= 0.0:
        status = 5
    return dict(P=P, H0=H0, H=H, Hmin=H.min(), iters=it, status=status, X=X, Y=Y, hx=hx, hy=hy)
