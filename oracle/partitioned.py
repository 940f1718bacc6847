"""Oracle (test infrastructure): the partitioned PAQIF solve of one long band
system (Sec. 2.1 eqs. 15-18 and Sec. 2.2 "PAQIF method", Steps 1-7).

Only tests/, the smoke check and the benchmark's CPU leg use this module.

The system of order N (half-bandwidth beta = q, band layout of the rest of
the oracle) is cut into r consecutive blocks along the diagonal; block m owns
rows p_m .. p_{m+1}-1 with p_m = floor(m N / r).  L0^(m) is the block's own
diagonal block, L-^(m) / L+^(m) the q x q couplings of its first / last q
rows to the last q unknowns of block m-1 / the first q of block m+1
(eq. 15).  Per block (dense matrices; small sizes only):

  Step 1  L0 = W0 Z0 by the centre-out AQIF factorisation (the oracle's C
          routine, Sec. 2.2);
  Step 2  W0 Y = F;
  Step 3  the inverse of the 2q x 2q block of W0 on the outer rows/columns
          (first q and last q): span{e_i, e_{n-i+1}}, i <= q, is invariant
          under W0 (Sec. 2.1), so the coupling terms of F* (which live on
          those rows only, eq. 18) change Y only there, by that inverse
          (eq. 31);
  Step 4  the first and last q equations of Z0 U = Y* of every block
          (the outer rows of Z0 vanish on the inner columns, eq. 33) form the
          reduced system R_d U_d = F_d in U_F^(m), U_L^(m) (eq. 35);
  Step 5  projection of U_F, U_L onto u >= 0 (bounded rows; CLIP only);
  Step 6  the inner rows: Z0* U_M = Y_M - (outer columns of Z0) U_o (eq. 38);
  Step 7  projection of U_M (CLIP only).

Reading: the paper solves R_d through the normal equations R_d^T R_d and a
Cholesky factorisation (eq. 37); that squares the condition number and has
the same solution, so the default here is a direct dense solve of R_d; the
normal equations are kept as an option (``reduced="normal"``) and a pin
checks that both agree.  The projection is componentwise max(0, .) on
bounded rows, as for the unpartitioned oracle.  Pins:
tests/test_oracle_partitioned.py.
"""
import numpy as np
import scipy.linalg as sla

from . import CLIP, LINEAR, aqif_factor_dense


def block_starts(N, r):
    """p_0 .. p_r with p_m = floor(m N / r)."""
    return [(m * N) // r for m in range(r + 1)]


def entry(band, i, j):
    """a(i, j) of the band matrix (0 outside the band or the matrix)."""
    N, w = band.shape
    q = (w - 1) // 2
    if not (0 <= i < N and 0 <= j < N) or abs(j - i) > q:
        return 0.0
    return float(band[i, j - i + q])


def dense(band):
    N, w = band.shape
    q = (w - 1) // 2
    A = np.zeros((N, N))
    for i in range(N):
        for d in range(-q, q + 1):
            if 0 <= i + d < N:
                A[i, i + d] = band[i, d + q]
    return A


def _block_band(band, p0, p1):
    """L0^(m): the rows p0..p1-1 with their columns outside the block
    dropped (the band layout ignores columns outside [0, n))."""
    q = (band.shape[1] - 1) // 2
    b = band[p0:p1].copy()
    n = p1 - p0
    for i in range(n):
        for d in range(-q, q + 1):
            if not 0 <= i + d < n:
                b[i, d + q] = 0.0
    return b


def solve_partitioned(band, f, r, bounded=None, mode=LINEAR, reduced="direct"):
    """Steps 1-7.  Returns u (N).  Every block needs at least 2q+1 rows."""
    band = np.asarray(band, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    N, w = band.shape
    q = (w - 1) // 2
    p = block_starts(N, r)
    if min(p[m + 1] - p[m] for m in range(r)) < 2 * q + 1:
        raise ValueError("every block needs at least 2q+1 rows")
    bnd = np.ones(N, dtype=bool) if bounded is None else np.asarray(bounded).astype(bool)

    blocks = []
    for m in range(r):
        n = p[m + 1] - p[m]
        W, Z, st = aqif_factor_dense(_block_band(band, p[m], p[m + 1]))   # Step 1
        if st != 0:
            raise ZeroDivisionError("zero pivot in block %d" % m)
        Y = np.linalg.solve(W, f[p[m]:p[m + 1]])                        # Step 2
        o = list(range(q)) + list(range(n - q, n))
        Winv = np.linalg.inv(W[np.ix_(o, o)])                             # Step 3
        blocks.append(dict(n=n, W=W, Z=Z, Y=Y, o=o, Winv=Winv))

    # Step 4: reduced system in (U_F^(1), U_L^(1), ..., U_F^(r), U_L^(r))
    K = 2 * q * r
    R = np.zeros((K, K))
    Fd = np.zeros(K)
    for m, B in enumerate(blocks):
        rows = slice(2 * q * m, 2 * q * (m + 1))
        R[rows, rows] = B["Z"][np.ix_(B["o"], B["o"])]
        Fd[rows] = B["Y"][B["o"]]
        # coupling of the block's first q rows to U_L^(m-1) (L-) and of its
        # last q rows to U_F^(m+1) (L+), moved through W0's outer inverse
        if m > 0:
            Lm = np.array([[entry(band, p[m] + i, p[m] - q + j) for j in range(q)]
                           for i in range(q)])
            cols = slice(2 * q * (m - 1) + q, 2 * q * m)
            R[rows, cols] += B["Winv"][:, :q] @ Lm
        if m < r - 1:
            Lp = np.array([[entry(band, p[m + 1] - q + i, p[m + 1] + j) for j in range(q)]
                           for i in range(q)])
            cols = slice(2 * q * (m + 1), 2 * q * (m + 1) + q)
            R[rows, cols] += B["Winv"][:, q:] @ Lp
    if reduced == "normal":
        Ud = sla.cho_solve(sla.cho_factor(R.T @ R), R.T @ Fd)
    else:
        Ud = np.linalg.solve(R, Fd)

    u = np.zeros(N)
    for m, B in enumerate(blocks):
        n, o = B["n"], B["o"]
        uo = Ud[2 * q * m:2 * q * (m + 1)].copy()
        go = [p[m] + i for i in o]
        if mode == CLIP:                                                  # Step 5
            uo = np.where(bnd[go], np.maximum(uo, 0.0), uo)
        inner = list(range(q, n - q))
        Z = B["Z"]
        rhs = B["Y"][inner] - Z[np.ix_(inner, o)] @ uo
        um = np.linalg.solve(Z[np.ix_(inner, inner)], rhs)                # Step 6
        gi = [p[m] + i for i in inner]
        if mode == CLIP:                                                  # Step 7
            um = np.where(bnd[gi], np.maximum(um, 0.0), um)
        u[go] = uo
        u[gi] = um
    return u
