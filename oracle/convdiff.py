"""Oracle (test infrastructure): the linear convection-diffusion workload of
the numerical-results section, solved by line relaxation with AQIF line
solves.

Problem (Example 1 with the linear case study of the numerical results):
(a u)_x + (b u)_y - eps (u_xx + u_yy) = f on [-1, 1]^2, Dirichlet data from
the exact solution u = x^4 + y^4, eps = 1e-6.  The paper leaves a and b
unspecified; constant a = b = 1 is used (the kappa-scheme derivation assumes
a constant positive a).

Discretisation (Sec. 3.1 kappa-schemes, eqs. 40-42): on a uniform (n x n)-node grid,
h = 2/(n-1), node (i, j) at (x_i, y_j); for a > 0 the convective term is the
flux difference a (u_{i+1/2} - u_{i-1/2}) / h with the kappa interface value
u_{i+1/2} = u_i + (1+kappa)/4 (u_{i+1} - u_i) + (1-kappa)/4 (u_i - u_{i-1});
at the first interior node next to the inflow boundary (i = 1) the missing
u_{-1} is the linear extrapolation 2 u_0 - u_1.
Diffusion is the 5-point Laplacian.  Same in y with b.

Iteration (line splitting as a defect correction): a half-step solves, on
every line of one direction at once, M sigma = f - L_h u with M the line's
whole operator along the line (kappa convection and diffusion; lower
dominant, so the interlocking factorisation's 2 x 2 pivots stay regular)
plus the diagonal of the across-line part, then u += omega sigma; x-lines
and y-lines alternate.  At the fixed point L_h u = f.  Pins: tests/test_oracle_convdiff.py.

Distributive line relaxation (Ls3 of Sec. 3.1, eqs. 51-54, the "kappa-distributive"
splitting): the change of a node is distributed, u_ij += s_ij - (s_{i+-1,j}
+ s_{i,j+-1})/4 (eq. 51), so a line solves for ghost changes s* whose
distributed pattern cancels the line's defect: row (i, l) of the line matrix
is L_h applied to the pattern of a unit ghost change at node (k, l), read at
(i, l).  The paper prints the resulting five-band coefficients in a garbled
form; here the matrix is that definition evaluated (its half-bandwidth is 3).
Lines of one direction are taken in two colours (odd, then even line
indices), since neighbouring lines' patterns overlap.
"""
import numpy as np
import scipy.linalg as sla


def grid(n):
    x = np.linspace(-1.0, 1.0, n)
    return x, 2.0 / (n - 1)


def exact(n):
    x, _ = grid(n)
    return x[:, None] ** 4 + x[None, :] ** 4


def rhs(n, eps, a=1.0, b=1.0):
    """f = a u_x + b u_y - eps Lap u for u = x^4 + y^4 (a, b constant)."""
    x, _ = grid(n)
    X, Y = x[:, None], x[None, :]
    return a * 4 * X ** 3 + b * 4 * Y ** 3 - eps * (12 * X ** 2 + 12 * Y ** 2)


def start(n):
    """Initial iterate: exact boundary values, zero inside."""
    u = exact(n)
    u[1:-1, 1:-1] = 0.0
    return u


def _conv_1d(u, axis, kappa, c, h):
    """c (u_{i+1/2} - u_{i-1/2}) / h along `axis` at interior nodes (kappa
    interface values)."""
    v = np.moveaxis(u, axis, 0)
    n = v.shape[0]
    out = np.zeros_like(v)
    i = np.arange(2, n - 1)
    d0 = v[i] - v[i - 1]          # u_i - u_{i-1}
    dp = v[i + 1] - v[i]          # u_{i+1} - u_i
    dm = v[i - 1] - v[i - 2]      # u_{i-1} - u_{i-2}
    up = v[i] + (1 + kappa) / 4 * dp + (1 - kappa) / 4 * d0      # u_{i+1/2}
    um = v[i - 1] + (1 + kappa) / 4 * d0 + (1 - kappa) / 4 * dm  # u_{i-1/2}
    out[2:n - 1] = c * (up - um) / h
    # first interior node: the missing u_{-1} is the linear extrapolation
    # 2 u_0 - u_1 (a ghost node), so u_{1/2} = (u_0 + u_1)/2
    up1 = v[1] + (1 + kappa) / 4 * (v[2] - v[1]) + (1 - kappa) / 4 * (v[1] - v[0])
    out[1] = c * (up1 - 0.5 * (v[0] + v[1])) / h
    return np.moveaxis(out, 0, axis)


def operator(u, kappa, eps, a=1.0, b=1.0):
    """L_h u at the interior nodes (zero on the boundary)."""
    n = u.shape[0]
    _, h = grid(n)
    out = _conv_1d(u, 0, kappa, a, h) + _conv_1d(u, 1, kappa, b, h)
    lap = np.zeros_like(u)
    lap[1:-1, 1:-1] = (u[2:, 1:-1] + u[:-2, 1:-1] + u[1:-1, 2:] + u[1:-1, :-2]
                       - 4 * u[1:-1, 1:-1]) / h ** 2
    out = out - eps * lap
    out[0, :] = out[-1, :] = out[:, 0] = out[:, -1] = 0.0
    return out


def defect(u, f, kappa, eps, a=1.0, b=1.0):
    r = f - operator(u, kappa, eps, a, b)
    r[0, :] = r[-1, :] = r[:, 0] = r[:, -1] = 0.0
    return r


def line_band(n, axis, l, kappa, eps, a=1.0, b=1.0):
    """The line operator M of line l (n-2 interior unknowns), as a band with
    half-bandwidth 2 (rows x 5, column s -> offset s-2): the whole
    convection and diffusion along the line (the kappa stencil of
    _conv_1d: u_{i+1} (1+k)/4, u_i (3-3k)/4, u_{i-1} (3k-5)/4, u_{i-2}
    (1-k)/4, times c/h; at the first interior node, with the ghost value,
    u_2 (1+k)/4, u_1 (1-k)/2, u_0 -(3-k)/4) plus
    the diagonal of the across-line part; entries on boundary nodes are
    left out (the correction vanishes there)."""
    _, h = grid(n)
    c_al, c_ac = (a, b) if axis == 0 else (b, a)
    m = n - 2
    band = np.zeros((m, 5))
    k = kappa
    across = c_ac / h * ((3 - 3 * k) / 4 if l >= 2 else (1 - k) / 2) + 2 * eps / h ** 2
    for r in range(m):
        i = r + 1
        if i >= 2:
            coef = {1: (1 + k) / 4, 0: (3 - 3 * k) / 4, -1: (3 * k - 5) / 4, -2: (1 - k) / 4}
        else:  # ghost u_{-1} = 2 u_0 - u_1
            coef = {1: (1 + k) / 4, 0: (1 - k) / 2, -1: -(3 - k) / 4}
        row = np.zeros(5)
        for off, cv in coef.items():
            row[off + 2] += c_al / h * cv
        row[1] += -eps / h ** 2
        row[2] += 2 * eps / h ** 2 + across
        row[3] += -eps / h ** 2
        for s in range(5):
            if not (0 <= r + s - 2 < m):
                row[s] = 0.0
        band[r] = row
    return band


def _band_to_ab(band):
    """(m x 5, offsets -2..2) -> scipy solve_banded layout (l = u = 2)."""
    m = band.shape[0]
    ab = np.zeros((5, m))
    for s in range(5):
        off = s - 2           # column j = i + off
        for i in range(m):
            j = i + off
            if 0 <= j < m:
                ab[2 + i - j, j] = band[i, s]
    return ab


def half_step(u, f, axis, kappa, eps, omega, a=1.0, b=1.0):
    """Solve M sigma = defect on every line of `axis` (x-lines: axis 0 runs
    along x), then u += omega sigma."""
    n = u.shape[0]
    r = defect(u, f, kappa, eps, a, b)
    un = u.copy()
    for l in range(1, n - 1):
        ab = _band_to_ab(line_band(n, axis, l, kappa, eps, a, b))
        rl = r[1:-1, l] if axis == 0 else r[l, 1:-1]
        sig = sla.solve_banded((2, 2), ab, rl)
        if axis == 0:
            un[1:-1, l] += omega * sig
        else:
            un[l, 1:-1] += omega * sig
    return un


def solve(n, kappa, eps=1e-6, omega=1.0, tol=1e-10, max_iter=500, a=1.0, b=1.0):
    """Alternate x- and y-line half-steps until max |f - L_h u| <= tol max|f|
    (checked after each full iteration).  Returns u, iterations, the final
    defect norm and the max / L1 / L2 errors against x^4 + y^4 (relative to
    the exact solution's norms, interior nodes)."""
    f = rhs(n, eps, a, b)
    u = start(n)
    fmax = np.abs(f[1:-1, 1:-1]).max()
    it = 0
    res = np.inf
    for it in range(1, max_iter + 1):
        u = half_step(u, f, 0, kappa, eps, omega, a, b)
        u = half_step(u, f, 1, kappa, eps, omega, a, b)
        res = np.abs(defect(u, f, kappa, eps, a, b)).max()
        if res <= tol * fmax:
            break
    e = (u - exact(n))[1:-1, 1:-1]
    ue = exact(n)[1:-1, 1:-1]
    errs = dict(linf=np.abs(e).max() / np.abs(ue).max(),
                l1=np.abs(e).sum() / np.abs(ue).sum(),
                l2=np.sqrt((e ** 2).sum() / (ue ** 2).sum()))
    return dict(u=u, iters=it, defect=res, fmax=fmax, **errs)


def pattern(n, node):
    """Distributed change of a unit ghost change at an interior node."""
    d = np.zeros((n, n))
    i, j = node
    d[i, j] = 1.0
    for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        if 1 <= i + di <= n - 2 and 1 <= j + dj <= n - 2:
            d[i + di, j + dj] -= 0.25
    return d


def ls3_line_matrix(n, axis, l, kappa, eps, a=1.0, b=1.0):
    """(n-2) x (n-2) matrix of line l: column k = L_h(pattern at the line's
    node k+1) on the line's nodes."""
    m = n - 2
    A = np.zeros((m, m))
    for k in range(m):
        node = (k + 1, l) if axis == 0 else (l, k + 1)
        col = operator(pattern(n, node), kappa, eps, a, b)
        A[:, k] = col[1:-1, l] if axis == 0 else col[l, 1:-1]
    return A


def ls3_half_step(u, f, axis, color, kappa, eps, omega, a=1.0, b=1.0):
    """Lines of one direction and colour (line index parity): ghost changes
    from the line matrices, then u += omega * (distributed changes)."""
    n = u.shape[0]
    r = defect(u, f, kappa, eps, a, b)
    g = np.zeros_like(u)
    for l in range(1, n - 1):
        if l % 2 != color:
            continue
        rl = r[1:-1, l] if axis == 0 else r[l, 1:-1]
        s = np.linalg.solve(ls3_line_matrix(n, axis, l, kappa, eps, a, b), rl)
        if axis == 0:
            g[1:-1, l] = s
        else:
            g[l, 1:-1] = s
    du = g.copy()
    du[1:, :] -= 0.25 * g[:-1, :]
    du[:-1, :] -= 0.25 * g[1:, :]
    du[:, 1:] -= 0.25 * g[:, :-1]
    du[:, :-1] -= 0.25 * g[:, 1:]
    du[0, :] = du[-1, :] = du[:, 0] = du[:, -1] = 0.0
    return u + omega * du


def ls3_iteration(u, f, kappa, eps, omega, a=1.0, b=1.0):
    """One iteration: x-lines (odd, even), then y-lines (odd, even)."""
    for axis in (0, 1):
        for color in (1, 0):
            u = ls3_half_step(u, f, axis, color, kappa, eps, omega, a, b)
    return u


def solve_ls3(n, kappa, eps=1e-6, omega=1.0, tol=1e-10, max_iter=500, a=1.0, b=1.0):
    """Ls3 iterations until max |f - L_h u| <= tol max|f|."""
    f = rhs(n, eps, a, b)
    u = start(n)
    fmax = np.abs(f[1:-1, 1:-1]).max()
    it, res = 0, np.inf
    for it in range(1, max_iter + 1):
        u = ls3_iteration(u, f, kappa, eps, omega, a, b)
        res = np.abs(defect(u, f, kappa, eps, a, b)).max()
        if res <= tol * fmax:
            break
    return dict(u=u, iters=it, defect=res, fmax=fmax)


# ---------------------------------------------------------------------------
# The paper's x-line splittings Ls0 and Ls1 (Sec. 3.1, eqs. 48-49): the
# forward x-line splitting L = L+ + L0 + L- with L0 the implicit operator of
# line j, L+ the upstream line(s) at their new values, L- the rest at the old
# ones.  Written as a defect correction: L0 sigma = f - L_h u (u with the
# lines already swept at their new values), u += omega sigma.
# ---------------------------------------------------------------------------

def split_weight(which, kappa):
    """Implicit weight of the x-upwind difference (u_i - u_{i-1}) a/h in L0:
    Ls1 (eq. 49) keeps the first-order upwind part (2 - kappa)/2, Ls0 (eq. 48)
    also the "positive" part of the upstream kappa term: (2 - kappa)/2 +
    (1 - kappa)/4."""
    if which == 1:
        return 0.5 * (2.0 - kappa)
    if which == 0:
        return 0.5 * (2.0 - kappa) + 0.25 * (1.0 - kappa)
    raise ValueError("which must be 0 (Ls0) or 1 (Ls1)")


def split_line_band(n, l, which, kappa, eps, a=1.0, b=1.0):
    """L0 of x-line l (n-2 interior unknowns) as a half-bandwidth-2 band
    (rows x 5, column s -> offset s-2): u_{i-1} -eps/h^2 - w a/h, u_i
    w a/h + 4 eps/h^2 + (the line's own y-convection coefficient), u_{i+1}
    -eps/h^2, w = split_weight(which, kappa).  The printed L0 has no b terms;
    the y-convection's coefficient of u_{i,j} itself (b/h (3-3kappa)/4, next
    to the inflow boundary (1-kappa)/2) is kept implicit like the diffusion
    diagonal; its upstream terms act through L+ (new values)."""
    _, h = grid(n)
    m = n - 2
    w = split_weight(which, kappa)
    own_y = b / h * ((3 - 3 * kappa) / 4 if l >= 2 else (1 - kappa) / 2)
    band = np.zeros((m, 5))
    for r in range(m):
        if r >= 1:
            band[r, 1] = -eps / h ** 2 - w * a / h
        band[r, 2] = w * a / h + 4 * eps / h ** 2 + own_y
        if r <= m - 2:
            band[r, 3] = -eps / h ** 2
    return band


def split_half_step(u, f, which, color, kappa, eps, omega, a=1.0, b=1.0):
    """The x-lines of one colour (line index parity) at once: L0 sigma = the
    defect on each, then u += omega sigma on those lines."""
    n = u.shape[0]
    r = defect(u, f, kappa, eps, a, b)
    un = u.copy()
    for l in range(1, n - 1):
        if l % 2 != color:
            continue
        ab = _band_to_ab(split_line_band(n, l, which, kappa, eps, a, b))
        un[1:-1, l] += omega * sla.solve_banded((2, 2), ab, r[1:-1, l])
    return un


def split_iteration(u, f, which, kappa, eps, omega, a=1.0, b=1.0, lexicographic=False):
    """One sweep over the x-lines: odd lines, then even ones (both colours see
    the other's latest values); lexicographic=True sweeps j = 1, 2, ... one
    line at a time as the paper's forward ordering does."""
    n = u.shape[0]
    if not lexicographic:
        for color in (1, 0):
            u = split_half_step(u, f, which, color, kappa, eps, omega, a, b)
        return u
    for l in range(1, n - 1):
        r = defect(u, f, kappa, eps, a, b)
        ab = _band_to_ab(split_line_band(n, l, which, kappa, eps, a, b))
        u = u.copy()
        u[1:-1, l] += omega * sla.solve_banded((2, 2), ab, r[1:-1, l])
    return u


def solve_split(n, which, kappa, eps=1e-6, omega=1.0, tol=1e-10, max_iter=500, a=1.0, b=1.0,
                lexicographic=False):
    """Ls0 (which = 0) or Ls1 (which = 1) sweeps until max |f - L_h u| <= tol
    max|f|."""
    f = rhs(n, eps, a, b)
    u = start(n)
    fmax = np.abs(f[1:-1, 1:-1]).max()
    it, res = 0, np.inf
    for it in range(1, max_iter + 1):
        u = split_iteration(u, f, which, kappa, eps, omega, a, b, lexicographic)
        res = np.abs(defect(u, f, kappa, eps, a, b)).max()
        if res <= tol * fmax or not np.isfinite(res):
            break
    return dict(u=u, iters=it, defect=res, fmax=fmax)
