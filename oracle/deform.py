"""Oracle (test infrastructure): elastic deformation kernels and sums, FP64.

Line contact, Sec. 3.3.1 "Film thickness calculation", case 1: the
deformation is -(1/pi) times the integral of ln|x - x'| P(x') over the
contact, with P piecewise constant on cells of width h centred at the grid
nodes.  The cell integral has a closed form: the integral of ln|t| over
[d - h/2, d + h/2] equals F(d + h/2) - F(d - h/2) with F(t) = t ln|t| - t and
F(0) = 0.

Readings: the printed cell formula uses |x+|(ln|x+| - 1) - |x-|(ln|x-| - 1),
which gives a zero self term and flips sign for negative offsets; the exact
antiderivative F above is used instead (pinned against quadrature).  The
factor 1/pi is applied once (it is written in the continuous integral and
in the discrete sum but not in the final film-thickness formula).

Point contact, case 2: (2/pi^2) times the integral of P/|r - r'|; the cell
integral over a square cell is the asinh expression of the paper, checked
here against numerical quadrature.  The factor 2/pi^2 is applied once.
"""
import numpy as np


def line_cell_integral(d, h):
    """Integral of ln|t| for t in [d - h/2, d + h/2] (vectorised)."""
    d = np.asarray(d, dtype=np.float64)

    def F(t):
        at = np.abs(t)
        out = np.zeros_like(t)
        nz = at > 0
        out[nz] = t[nz] * np.log(at[nz]) - t[nz]
        return out

    return F(d + 0.5 * h) - F(d - 0.5 * h)


def line_kernel(N, h):
    """Kernel coefficients k[m] = -(1/pi) * cell integral at offset m*h,
    m = 0..N-1; the deformation matrix is K[i, j] = k[|i - j|]."""
    m = np.arange(N, dtype=np.float64)
    return -line_cell_integral(m * h, h) / np.pi


def line_matrix(N, h):
    k = line_kernel(N, h)
    idx = np.abs(np.arange(N)[:, None] - np.arange(N)[None, :])
    return k[idx]


def line_deformation(P, h):
    """H_el = K P for P of shape (N,) or (N, B) (columns = instances)."""
    P = np.asarray(P, dtype=np.float64)
    K = line_matrix(P.shape[0], h)
    return K @ P


def point_cell_integral(dx, dy, hx, hy):
    """Integral of 1/sqrt((dx - x')^2 + (dy - y')^2) over the cell
    [-hx/2, hx/2] x [-hy/2, hy/2] (closed form, asinh terms)."""
    dx = np.asarray(dx, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    xp, xm = dx + 0.5 * hx, dx - 0.5 * hx
    yp, ym = dy + 0.5 * hy, dy - 0.5 * hy

    def term(a, b):
        # |a| asinh(b/a) with the a -> 0 limit 0
        out = np.zeros(np.broadcast(a, b).shape)
        a_b, b_b = np.broadcast_arrays(a, b)
        nz = a_b != 0
        out[nz] = np.abs(a_b[nz]) * np.arcsinh(b_b[nz] / a_b[nz])
        return out

    return (term(xp, yp) + term(yp, xp) - term(xm, yp) - term(yp, xm)
            - term(xp, ym) - term(ym, xp) + term(xm, ym) + term(ym, xm))


def point_kernel(Nx, Ny, hx, hy):
    """k2[a, b] = (2/pi^2) * cell integral at offset (a*hx, b*hy)."""
    a = np.arange(Nx, dtype=np.float64)[:, None] * hx
    b = np.arange(Ny, dtype=np.float64)[None, :] * hy
    return 2.0 / np.pi ** 2 * point_cell_integral(a, b, hx, hy)


def point_deformation(P, hx, hy):
    """H_el[i, j] = sum_{i', j'} k2[|i-i'|, |j-j'|] P[i', j'] (direct sum).

    P has shape (Nx, Ny).  Evaluated as, for every row offset, a dense
    Toeplitz product along y (matmul is the library primitive)."""
    P = np.asarray(P, dtype=np.float64)
    Nx, Ny = P.shape
    k2 = point_kernel(Nx, Ny, hx, hy)
    jj = np.abs(np.arange(Ny)[:, None] - np.arange(Ny)[None, :])
    H = np.zeros((Nx, Ny))
    for d in range(Nx):
        T = k2[d][jj]                 # Ny x Ny Toeplitz block for row offset d
        Q = P @ T                     # Q[i', j] = sum_j' T[j, j'] P[i', j'] (T symmetric)
        if d == 0:
            H += Q
        else:
            H[d:, :] += Q[:-d, :]     # i = i' + d
            H[:-d, :] += Q[d:, :]     # i = i' - d
    return H
