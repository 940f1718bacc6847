"""Pins of the convection-diffusion oracle (CPU).

  * the kappa-scheme operator reproduces the continuous operator exactly on
    a linear field at every interior node and on a quadratic field away from
    the inflow boundary (the ghost node is a linear extrapolation), for every
    kappa: a wrong coefficient, sign or index in the stencil fails it;
  * the line relaxation's fixed point is the discrete solution: it equals a
    direct sparse solve of the operator assembled column by column from unit
    vectors (brute force, no line structure);
  * grid convergence against u = x^4 + y^4: order >= 1.9 in the max norm
    from 17 to 33 to 65 nodes per side, for kappa = 0, 1/3, -1.
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
