"""Pins of the oracle's banded AQIF / LCP against things other than itself.

  * LAPACK banded LU (scipy.linalg.solve_banded) and dense LU on the same
    systems, symmetric and non-symmetric, odd and even orders, tiny orders;
  * the factor shapes of Sec. 2.2 (unit "hourglass" W0, "butterfly" Z0, and
    the banded index ranges: Z0 rows with 2q+1 entries, W0 columns with 2q),
    and the reconstruction W0 Z0 = A;
  * the LCP of Sec. 2.1 eq. (14): brute force over all 2^n active sets on
    small systems (unique solution for these P-matrices), the projected SOR
    iteration of Sec. 3.2 (Cryer), the QP characterisation (bound-constrained
    minimisation of 1/2 u'Au - b'u by scipy), and the complementarity
    certificate at full size;
  * the start sweeps (projected Jacobi, a starting active set of the exact
    LCP): one sweep against its closed form, several against the same
    iteration written with the dense matrix, many against the LCP solution
    (their fixed point for a strictly diagonally dominant matrix).
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.optimize as so

import oracle
import synth


def dense(band):
    n, w = band.shape
    q = (w - 1) // 2
    A = np.zeros((n, n))
    for i in range(n):
        for d in range(-q, q + 1):
            if 0 <= i + d < n:
                A[i, i + d] = band[i, d + q]
    return A


def nonsym_band(n, q, seed):
    rng = np.random.default_rng(seed)
    band = rng.uniform(-1, 1, size=(n, 2 * q + 1))
    for i in range(n):
        for d in range(-q, q + 1):
            if not 0 <= i + d < n:
                band[i, d + q] = 0.0
    band[:, q] = np.abs(band).sum(axis=1) + rng.uniform(0.5, 1.5, size=n)
    return band, rng.normal(size=n)


def lapack_banded(band, f):
    n, w = band.shape
    q = (w - 1) // 2
    ab = np.zeros((2 * q + 1, n))
    for i in range(n):
        for d in range(-q, q + 1):
            j = i + d
            if 0 <= j < n:
                ab[q + i - j, j] = band[i, d + q]
    return sl.solve_banded((q, q), ab, f)


SIZES = [1, 2, 3, 4, 5, 6, 7, 8, 9, 15, 16, 17, 31, 64, 65, 200, 513]


@pytest.mark.parametrize("q", [1, 2, 3, 4, 8])
def test_aqif_matches_lapack(q):
    for n in SIZES:
        for band, f in (synth.lcp_system(n, q, 0, n), nonsym_band(n, q, n + 100 * q)):
            x, st = oracle.aqif_solve(band, f)
            assert st == oracle.OK
            xr = lapack_banded(band, f)
            xd = np.linalg.solve(dense(band), f)
            scale = max(1.0, np.abs(xr).max())
            assert np.abs(x - xr).max() / scale < 1e-13, (q, n)
            assert np.abs(x - xd).max() / scale < 1e-13, (q, n)


def _w_zero_expected(n):
    """Zero pattern of W0 (Sec. 2.2, definition of w_ij), 1-based in the
    paper, for even n: for 1 <= j <= n/2, w_ij = 0 for j+1 <= i <= n-j+1;
    for n/2+1 <= j <= n, w_ij = 0 for n-j+1 <= i <= j-1; w_jj = 1."""
    Zm = np.zeros((n, n), dtype=bool)
    h = n // 2
    for j in range(1, n + 1):
        if j <= h:
            rows = range(j + 1, n - j + 2)
        else:
            rows = range(n - j + 1, j)
        for i in rows:
            if i != j and 1 <= i <= n:
                Zm[i - 1, j - 1] = True
    return Zm


def _z_zero_expected(n):
    """Zero pattern of Z0: for 1 <= i <= (n-1)/2 (floor), z_ij = 0 for
    i+1 <= j <= n-i; for n+1-n/2 <= i <= n, z_ij = 0 for n-i+2 <= j <= i-1."""
    Zm = np.zeros((n, n), dtype=bool)
    for i in range(1, (n - 1) // 2 + 1):
        for j in range(i + 1, n - i + 1):
            Zm[i - 1, j - 1] = True
    for i in range(n + 1 - n // 2, n + 1):
        for j in range(n - i + 2, i):
            Zm[i - 1, j - 1] = True
    return Zm


@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_factor_shapes_and_reconstruction(q):
    for n in [2, 4, 6, 8, 10, 16, 24, 3, 5, 9, 17]:
        band, _ = nonsym_band(n, q, 7 * n + q)
        A = dense(band)
        W, Z, st = oracle.aqif_factor_dense(band)
        assert st == oracle.OK
        assert np.abs(W @ Z - A).max() <= 1e-14 * np.abs(A).max() * n
        assert np.allclose(np.diag(W), 1.0)
        if n % 2 == 0:
            assert (W[_w_zero_expected(n)] == 0).all()
            assert (Z[_z_zero_expected(n)] == 0).all()
        # banded index ranges: Z0 rows have at most 2q+1 entries, W0 columns
        # at most 2q off-diagonal entries
        assert (np.count_nonzero(Z, axis=1) <= 2 * q + 1).all()
        assert (np.count_nonzero(W - np.eye(n), axis=0) <= 2 * q).all()


def test_pinned_rows_give_reduced_solve():
    q = 3
    for n in [7, 20, 41]:
        band, f = nonsym_band(n, q, n)
        rng = np.random.default_rng(n)
        pin = (rng.random(n) < 0.3).astype(np.uint8)
        x, st = oracle.aqif_solve(band, f, pin)
        assert st == oracle.OK
        A = dense(band)
        I = np.where(pin == 0)[0]
        xr = np.zeros(n)
        xr[I] = np.linalg.solve(A[np.ix_(I, I)], f[I])
        assert (x[pin == 1] == 0.0).all()
        assert np.abs(x - xr).max() < 1e-13 * max(1, np.abs(xr).max())


def brute_force_lcp(A, f, bounded=None):
    n = len(f)
    bnd = np.ones(n, dtype=bool) if bounded is None else bounded.astype(bool)
    idx = np.where(bnd)[0]
    sols = []
    for mask in itertools.product([0, 1], repeat=len(idx)):
        act = np.zeros(n, dtype=bool)
        act[idx[np.array(mask, dtype=bool)]] = True
        I = np.where(~act)[0]
        u = np.zeros(n)
        if len(I):
            u[I] = np.linalg.solve(A[np.ix_(I, I)], f[I])
        w = A @ u - f
        if (u[bnd] >= -1e-12).all() and (w[bnd] >= -1e-12).all() and \
                (np.abs(w[~bnd]) < 1e-10).all():
            sols.append((u, act))
    return sols


@pytest.mark.parametrize("q", [1, 2, 4])
def test_lcp_brute_force(q):
    for n in [1, 2, 3, 5, 8, 11]:
        for item in range(4):
            band, f = synth.lcp_system(n, q, 1, item)
            A = dense(band)
            sols = brute_force_lcp(A, f)
            assert len(sols) == 1
            r = oracle.lcp_solve(band, f, mode=oracle.EXACT)
            assert r["status"] == oracle.OK
            assert np.abs(r["u"] - sols[0][0]).max() < 1e-12
            assert (r["active"].astype(bool) == sols[0][1]).all() or \
                np.abs(r["u"][r["active"] != sols[0][1]]).max() < 1e-12


@pytest.mark.parametrize("q", [1, 2, 4])
def test_lcp_empty_start_reaches_the_same_solution(q):
    """The active-set iteration from the empty set (the textbook start) and
    from the sign of f reach the same, unique, solution; both agree with
    brute force on small systems and with each other at full size."""
    for n in [1, 2, 5, 11]:
        for item in range(3):
            band, f = synth.lcp_system(n, q, 1, item)
            sols = brute_force_lcp(dense(band), f)
            r0 = oracle.lcp_solve_start(band, f)
            assert r0["status"] == oracle.OK
            assert np.abs(r0["u"] - sols[0][0]).max() < 1e-12
    band, f = synth.lcp_system(4097, q, 0, 0)
    r0 = oracle.lcp_solve_start(band, f)
    r1 = oracle.lcp_solve(band, f, mode=oracle.EXACT)
    assert r0["status"] == oracle.OK and r1["status"] == oracle.OK
    assert (r0["active"] == r1["active"]).all()
    assert np.abs(r0["u"] - r1["u"]).max() <= 1e-13 * max(1.0, np.abs(r1["u"]).max())
    # a start equal to the solution's active set ends after one solve
    r2 = oracle.lcp_solve_start(band, f, start=r1["active"])
    assert r2["iters"] == 1 and (r2["active"] == r1["active"]).all()


@pytest.mark.parametrize("q", [1, 2, 4, 8])
def test_start_sweeps_one_sweep_closed_form(q):
    """From u = 0 one sweep gives f_i / a_ii, clipped at 0 on bounded rows."""
    band, f = nonsym_band(37, q, 5)
    bounded = (np.arange(37) % 3 != 0).astype(np.uint8)
    u = oracle.start_sweeps(band, f, bounded, 1)
    x = f / band[:, q]
    ref = np.where(bounded != 0, np.maximum(x, 0.0), x)
    assert np.array_equal(u, ref)
    assert np.array_equal(oracle.start_sweeps(band, f, bounded, 0), np.zeros(37))


@pytest.mark.parametrize("q", [1, 2, 4])
def test_start_sweeps_match_the_dense_iteration(q):
    """k sweeps u <- P(D^-1 (f - (A - D) u)) written with the dense matrix
    (P: clip at 0 on bounded rows), every sweep from the previous iterate
    only (Jacobi, not Gauss-Seidel)."""
    for n, k in [(1, 3), (2, 4), (9, 5), (40, 7)]:
        band, f = nonsym_band(n, q, 11 + n)
        bounded = (np.arange(n) % 4 != 1).astype(np.uint8)
        A = dense(band)
        D = np.diag(A)
        u = np.zeros(n)
        for _ in range(k):
            x = (f - (A - np.diag(D)) @ u) / D
            u = np.where(bounded != 0, np.maximum(x, 0.0), x)
        got = oracle.start_sweeps(band, f, bounded, k)
        assert np.abs(got - u).max() <= 1e-13 * max(1.0, np.abs(u).max()), (n, k)


@pytest.mark.parametrize("q", [2, 8])
def test_start_sweeps_converge_to_the_lcp_solution(q):
    """For a strictly diagonally dominant matrix the projected Jacobi
    iteration contracts, and its fixed point (u_i = max(0, (f_i - sum_{j!=i}
    a_ij u_j) / a_ii) on bounded rows, a_ii > 0) is the LCP's solution."""
    band, f = synth.lcp_system(300, q, 3, 0)
    bounded = (np.arange(300) % 5 != 2).astype(np.uint8)
    u = oracle.start_sweeps(band, f, bounded, 400)
    r = oracle.lcp_solve(band, f, bounded, mode=oracle.EXACT)
    assert r["status"] == oracle.OK
    assert np.abs(u - r["u"]).max() <= 1e-10 * max(1.0, np.abs(r["u"]).max())


def test_lcp_start_sets_rule():
    """The batch start rule with a size threshold: the systems with at
    least 0.7 (max_n // 2) elimination levels from the sweeps, the others
    from the sign of f; without one (frac = 0) every system from the
    sweeps; one sweep reproduces the sign start (positive diagonals)."""
    q = 2
    sizes = [1, 6, 40, 57, 60]
    offs, band, f = synth.lcp_batch(len(sizes), q, seed=3, sizes=sizes)
    bounded = (np.arange(int(offs[-1])) % 7 != 3).astype(np.uint8)
    sign = (bounded != 0) & (f <= 0.0)
    assert np.array_equal(oracle.lcp_start_sets(q, offs, band, f, bounded, k=0), sign)
    assert np.array_equal(oracle.lcp_start_sets(q, offs, band, f, bounded, k=1), sign)
    st = oracle.lcp_start_sets(q, offs, band, f, bounded, k=6, frac=0.7)
    band = band.reshape(-1, 2 * q + 1)
    for s, n in enumerate(sizes):  # levels 0 3 20 28 30; threshold int(0.7 * 30) = 21
        a, b = int(offs[s]), int(offs[s + 1])
        if n // 2 >= 21:
            u = oracle.start_sweeps(band[a:b], f[a:b], bounded[a:b], 6)
            assert np.array_equal(st[a:b], (bounded[a:b] != 0) & (u <= 0.0))
        else:
            assert np.array_equal(st[a:b], sign[a:b])
    st0 = oracle.lcp_start_sets(q, offs, band, f, bounded, k=6)
    for s, n in enumerate(sizes):
        a, b = int(offs[s]), int(offs[s + 1])
        u = oracle.start_sweeps(band[a:b], f[a:b], bounded[a:b], 6)
        assert np.array_equal(st0[a:b], (bounded[a:b] != 0) & (u <= 0.0))


def test_lcp_brute_force_with_free_rows():
    q = 2
    for item in range(6):
        n = 9
        band, f = synth.lcp_system(n, q, 2, item)
        bounded = (np.random.default_rng(item).random(n) < 0.6).astype(np.uint8)
        sols = brute_force_lcp(dense(band), f, bounded)
        assert len(sols) == 1
        r = oracle.lcp_solve(band, f, bounded=bounded, mode=oracle.EXACT)
        assert r["status"] == oracle.OK
        assert np.abs(r["u"] - sols[0][0]).max() < 1e-12
        assert not r["active"][bounded == 0].any()


def test_lcp_linear_and_clip_modes():
    band, f = synth.lcp_system(50, 4, 3, 0)
    A = dense(band)
    x = np.linalg.solve(A, f)
    r = oracle.lcp_solve(band, f, mode=oracle.LINEAR)
    assert np.abs(r["u"] - x).max() < 1e-13
    assert np.abs(r["w"]).max() < 1e-12
    r = oracle.lcp_solve(band, f, mode=oracle.CLIP)
    assert np.abs(r["u"] - np.maximum(x, 0)).max() < 1e-13
    assert np.abs(r["w"] - (A @ np.maximum(x, 0) - f)).max() < 1e-12


@pytest.mark.parametrize("q", [2, 4, 8])
def test_lcp_agrees_with_projected_sor_and_qp(q):
    band, f = synth.lcp_system(300, q, 4, q)
    r = oracle.lcp_solve(band, f, mode=oracle.EXACT)
    assert r["status"] == oracle.OK
    u_pgs, st, _ = oracle.lcp_pgs(band, f, omega=1.0, tol=1e-15)
    assert st == oracle.OK
    assert np.abs(r["u"] - u_pgs).max() < 1e-10
    A = dense(band)
    res = so.minimize(lambda u: 0.5 * u @ A @ u - f @ u, np.zeros(len(f)),
                      jac=lambda u: A @ u - f, method="L-BFGS-B",
                      bounds=[(0, None)] * len(f), options=dict(ftol=1e-15, gtol=1e-12,
                                                                maxiter=10000))
    assert np.abs(res.x - r["u"]).max() < 1e-6


def test_lcp_certificate_full_size():
    for q in (2, 4, 8):
        band, f = synth.lcp_system(4097, q, 0, 0)
        r = oracle.lcp_solve(band, f, mode=oracle.EXACT)
        assert r["status"] == oracle.OK
        u, w, a = r["u"], r["w"], r["active"]
        assert u.min() >= 0 and (u[a == 1] == 0).all()
        assert w.min() >= -1e-12 * np.abs(f).max()
        assert np.abs(u * w).max() <= 1e-12 * np.abs(f).max() * max(1, np.abs(u).max())
        # active-set iteration counts (context: a handful of solves)
        assert 2 <= r["iters"] <= 10


def test_zero_pivot_reported():
    band, f = synth.lcp_system(5, 2, 0, 0)
    band[2, :] = 0.0  # centre row of an odd system -> 1x1 pivot 0
    x, st = oracle.aqif_solve(band, f)
    assert st == oracle.ZERO_PIVOT
    band, f = synth.lcp_system(4, 1, 0, 0)
    band[1:3, :] = 0.0  # centre 2x2 block singular
    x, st = oracle.aqif_solve(band, f)
    assert st == oracle.ZERO_PIVOT


def test_planted_mistake_is_caught():
    """A wrong sign in one band entry (as a transposed operand would give on a
    non-symmetric matrix) must move the solution well beyond the tolerance."""
    band, f = nonsym_band(40, 3, 5)
    bad = band.copy()
    bad[20, 1] = -bad[20, 1]
    x_bad, _ = oracle.aqif_solve(bad, f)
    xr = lapack_banded(band, f)
    assert np.abs(x_bad - xr).max() > 1e-6
