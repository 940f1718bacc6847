"""Pins of the partitioned PAQIF oracle (CPU).

  * the invariance the method rests on (Sec. 2.1): W0 of a block maps the
    outer unit vectors (first and last q) into their own span, and the outer
    rows of Z0 vanish on the inner columns -- exact zeros;
  * linear mode: the partitioned solution is A^{-1} f of the whole system
    (numpy's dense solve), for ragged and even splits, odd and even block
    sizes, one block, and blocks of the minimum size 2q+1;
  * clip mode (Steps 5 and 7): equals an independent block elimination
    written with plain dense algebra -- the Schur complement of A on the
    outer unknowns of all blocks, solved and projected, then the inner
    unknowns from A_ii u_M = f_i - A_io u_o, projected -- no W0/Z0 anywhere;
  * the paper's normal equations (eq. 37) give the direct solution of R_d.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import partitioned as P


def _schur_clip(band, f, r, bounded):
    """Steps 4-7 by plain block elimination (independent of the AQIF)."""
    A = P.dense(band)
    N = A.shape[0]
    q = (band.shape[1] - 1) // 2
    p = P.block_starts(N, r)
    outer = []
    for m in range(r):
        outer += list(range(p[m], p[m] + q)) + list(range(p[m + 1] - q, p[m + 1]))
    inner = [i for i in range(N) if i not in set(outer)]
    Aoo, Aoi = A[np.ix_(outer, outer)], A[np.ix_(outer, inner)]
    Aio, Aii = A[np.ix_(inner, outer)], A[np.ix_(inner, inner)]
    S = Aoo - Aoi @ np.linalg.solve(Aii, Aio)
    g = f[outer] - Aoi @ np.linalg.solve(Aii, f[inner])
    uo = np.linalg.solve(S, g)
    uo = np.where(bounded[outer], np.maximum(uo, 0.0), uo)
    um = np.linalg.solve(Aii, f[inner] - Aio @ uo)
    um = np.where(bounded[inner], np.maximum(um, 0.0), um)
    u = np.zeros(N)
    u[outer] = uo
    u[inner] = um
    return u


@pytest.mark.parametrize("n,q", [(12, 2), (13, 2), (21, 4), (30, 4), (40, 8)])
def test_outer_span_invariant(n, q):
    band, _ = synth.long_system(n, q, seed=3)
    W, Z, st = oracle.aqif_factor_dense(band)
    assert st == 0
    o = list(range(q)) + list(range(n - q, n))
    i = list(range(q, n - q))
    assert np.all(W[np.ix_(i, o)] == 0.0)
    assert np.all(Z[np.ix_(o, i)] == 0.0)
    A = P.dense(band)
    assert np.abs(W @ Z - A).max() <= 1e-12 * np.abs(A).max()


CASES = [(60, 2, 4), (61, 2, 4), (97, 2, 7), (50, 2, 1), (5 * 7, 2, 7), (200, 4, 6),
         (203, 4, 5), (9 * 8, 4, 8), (300, 8, 5)]


@pytest.mark.parametrize("N,q,r", CASES)
def test_linear_is_the_direct_solution(N, q, r):
    band, f = synth.long_system(N, q, seed=N + r)
    u = P.solve_partitioned(band, f, r, mode=oracle.LINEAR)
    ref = np.linalg.solve(P.dense(band), f)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("N,q,r", CASES)
@pytest.mark.parametrize("masked", [False, True])
def test_clip_is_the_projected_block_elimination(N, q, r, masked):
    band, f = synth.long_system(N, q, seed=2 * N + r)
    rng = np.random.default_rng(N)
    bounded = rng.random(N) < 0.7 if masked else np.ones(N, dtype=bool)
    u = P.solve_partitioned(band, f, r, bounded=bounded.astype(np.uint8), mode=oracle.CLIP)
    ref = _schur_clip(band, f, r, bounded)
    assert np.abs(u - ref).max() <= 1e-11 * max(np.abs(ref).max(), 1.0)
    assert (u[bounded] >= 0).all()
    # the projection bites: some bounded rows are clipped (not the linear answer)
    lin = P.solve_partitioned(band, f, r, mode=oracle.LINEAR)
    assert (lin[bounded] < 0).any()


@pytest.mark.parametrize("N,q,r", [(60, 2, 4), (200, 4, 6)])
def test_normal_equations_agree(N, q, r):
    band, f = synth.long_system(N, q, seed=7)
    a = P.solve_partitioned(band, f, r, reduced="normal")
    b = P.solve_partitioned(band, f, r)
    assert np.abs(a - b).max() <= 1e-9 * np.abs(b).max()


def test_block_too_small_is_refused():
    band, f = synth.long_system(20, 2, seed=1)
    with pytest.raises(ValueError):
        P.solve_partitioned(band, f, 5)   # blocks of 4 < 2q+1 rows
