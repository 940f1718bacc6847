"""Pins of the convection-diffusion oracle (CPU).

  * the kappa-scheme operator reproduces the continuous operator exactly on
    a linear field at every interior node and on a quadratic field away from
    the inflow boundary (the ghost node is a linear extrapolation), for every
    kappa: a wrong coefficient, sign or index in the stencil fails it;
  * the line relaxation's fixed point is the discrete solution: it equals a
    direct sparse solve of the operator assembled column by column from unit
    vectors (brute force, no line structure);
  * grid convergence against u = x^4 + y^4: order >= 1.9 in the max norm
    from 17 to 33 to 65 nodes per side, for kappa = 0, 1/3, -1;
  * distributive line relaxation (Ls3): the line matrix has half-bandwidth 3
    (the pattern reaches one node either side of a stencil of offsets -2..1)
    and its entries equal the kappa stencil composed with the pattern by
    hand on a row far from the boundary; the iteration converges (slowly,
    as the paper warns) to the direct solution on 9 x 9 nodes.
  * x-line splittings Ls0 / Ls1: the implicit line operator L0 equals the
    coefficients printed in eqs. 48 / 49 (with b = 0, the terms the paper
    prints); the two-colour and the lexicographic sweeps converge, under-
    relaxed, to the direct solution.
The absolute errors of the paper's printed table are not reproduced (the
paper does not give a(x, y), b(x, y) nor its boundary closure): parity
unpinned there.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import convdiff as C

KAPPAS = [0.0, 1.0 / 3.0, -1.0]


@pytest.mark.parametrize("kappa", KAPPAS)
def test_operator_exact_on_low_degree_polynomials(kappa):
    n, eps, a, b = 21, 0.3, 1.0, 1.0   # a visible eps exercises the diffusion part
    x, h = C.grid(n)
    X, Y = x[:, None], x[None, :]
    lin = 1.0 + 2.0 * X - 3.0 * Y
    Lh = C.operator(lin, kappa, eps, a, b)
    assert np.abs(Lh[1:-1, 1:-1] - (a * 2.0 + b * (-3.0))).max() <= 1e-11
    quad = 1.0 + 2.0 * X - 3.0 * Y + X ** 2 - X * Y + 2.0 * Y ** 2
    Lh = C.operator(quad, kappa, eps, a, b)
    ref = a * (2.0 + 2 * X - Y) + b * (-3.0 - X + 4 * Y) - eps * (2.0 + 4.0)
    assert np.abs(Lh[2:-1, 2:-1] - ref[2:-1, 2:-1]).max() <= 1e-10


@pytest.mark.parametrize("kappa", KAPPAS)
def test_fixed_point_is_the_direct_solution(kappa):
    n, eps = 13, 1e-6
    f = C.rhs(n, eps)
    r = C.solve(n, kappa, eps=eps, tol=1e-13, max_iter=500)
    assert r["defect"] <= 1e-13 * r["fmax"]
    # assemble L_h on the interior unknowns column by column, boundary data
    # moved to the right-hand side
    m = n - 2
    ub = C.exact(n)
    ub[1:-1, 1:-1] = 0.0
    rhs = (f - C.operator(ub, kappa, eps))[1:-1, 1:-1].ravel()
    cols = []
    for k in range(m * m):
        e = np.zeros((n, n))
        e[1 + k // m, 1 + k % m] = 1.0
        cols.append(C.operator(e, kappa, eps)[1:-1, 1:-1].ravel())
    A = sp.csc_matrix(np.array(cols).T)
    u = spla.spsolve(A, rhs)
    assert np.abs(u - r["u"][1:-1, 1:-1].ravel()).max() <= 1e-10 * np.abs(u).max()


@pytest.mark.parametrize("kappa", KAPPAS)
def test_second_order_convergence(kappa):
    errs = [C.solve(n, kappa, tol=1e-12, max_iter=400)["linf"] for n in (17, 33, 65)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (orders >= 1.9).all(), (errs, orders)


@pytest.mark.parametrize("kappa", KAPPAS)
def test_ls3_line_matrix_band_and_stencil(kappa):
    n, eps, a, b = 15, 0.2, 1.0, 1.0
    _, h = C.grid(n)
    l = 6
    A = C.ls3_line_matrix(n, 0, l, kappa, eps, a, b)
    m = n - 2
    off = np.subtract.outer(np.arange(m), np.arange(m))      # row - column
    assert np.all(A[(off > 3) | (off < -2)] == 0.0)
    # interior row: along-line stencil c(-2..1) of the kappa scheme plus
    # diffusion, composed with the pattern (1 at the node, -1/4 either side);
    # across-line neighbours of the node get -1/4 through the across stencil
    k = kappa
    al = {-2: a / h * (1 - k) / 4, -1: a / h * (3 * k - 5) / 4 - eps / h ** 2,
          0: a / h * (3 - 3 * k) / 4 + 2 * eps / h ** 2, 1: a / h * (1 + k) / 4 - eps / h ** 2}
    ac = {-1: b / h * (3 * k - 5) / 4 - eps / h ** 2, 1: b / h * (1 + k) / 4 - eps / h ** 2}
    ac0 = b / h * (3 - 3 * k) / 4 + 2 * eps / h ** 2
    coef = dict(al)
    coef[0] = al[0] + ac0                   # the node's whole diagonal
    i = 7                                   # row of node i + 1 = 8
    for dc in range(-3, 3):
        ref = 0.0
        for s_, w in ((0, 1.0), (-1, -0.25), (1, -0.25)):
            ref += w * coef.get(dc + s_, 0.0)
        if dc == 0:
            ref -= 0.25 * (ac[-1] + ac[1])
        assert abs(A[i, i + dc] - ref) <= 1e-12 * max(1.0, abs(ref)), (dc, A[i, i + dc], ref)


@pytest.mark.parametrize("kappa", KAPPAS)
def test_ls3_converges_to_the_direct_solution(kappa):
    n = 9
    r = C.solve_ls3(n, kappa, tol=1e-11, max_iter=600)
    assert r["defect"] <= 1e-11 * r["fmax"]
    d = C.solve(n, kappa, tol=1e-13, max_iter=500)
    assert np.abs(r["u"] - d["u"]).max() <= 1e-9 * np.abs(d["u"]).max()


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("kappa", KAPPAS)
def test_split_line_operator_is_the_printed_one(which, kappa):
    """Interior and first rows of L0 against eq. 48 (Ls0) / eq. 49 (Ls1):
    u_{i-1}: -eps/h^2 - a/h w, u_i: a/h w + 4 eps/h^2, u_{i+1}: -eps/h^2 with
    w = (2-k)/2 + (1-k)/4 = (5-3k)/4 for Ls0 (printed as a/(4h)(5-3k) and
    a/h((2-k)/2 + (1-k)/4)) and w = (2-k)/2 for Ls1."""
    n, eps, a = 11, 0.05, 1.3
    _, h = C.grid(n)
    band = C.split_line_band(n, 4, which, kappa, eps, a, 0.0)
    k = kappa
    if which == 0:
        lo, di = -(eps / h ** 2 + a / (4 * h) * (5 - 3 * k)), a / h * ((2 - k) / 2 + (1 - k) / 4)
    else:
        lo, di = -a / h * (2 - k) / 2 - eps / h ** 2, a / h * (2 - k) / 2
    di += 4 * eps / h ** 2
    up = -eps / h ** 2
    for r in (3, 0, n - 3):
        ref = [0.0, lo if r > 0 else 0.0, di, up if r < n - 3 else 0.0, 0.0]
        assert np.abs(band[r] - np.array(ref)).max() <= 1e-12 * abs(di), (r, band[r], ref)
    # the y-convection's own coefficient joins the diagonal (b > 0)
    band_b = C.split_line_band(n, 4, which, kappa, eps, a, 0.7)
    assert abs(band_b[3, 2] - band[3, 2] - 0.7 / h * (3 - 3 * k) / 4) <= 1e-12 * abs(di)


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("kappa", KAPPAS)
def test_split_sweeps_converge_to_the_direct_solution(which, kappa):
    n = 13
    d = C.solve(n, kappa, tol=1e-13, max_iter=500)
    for lex in (False, True):
        r = C.solve_split(n, which, kappa, omega=0.7, tol=1e-12, max_iter=2000, lexicographic=lex)
        assert r["defect"] <= 1e-12 * r["fmax"], (lex, r["iters"])
        assert np.abs(r["u"] - d["u"]).max() <= 1e-10 * np.abs(d["u"]).max()
