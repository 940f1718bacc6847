"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no factorisation, no kernels, no EHL physics).  Every
array is produced on the host in FP64 from ``numpy.random.default_rng`` with a
seed list ``[workload, seed, item]``, so a single system of a batch can be
regenerated on its own.

Workloads (the paper publishes no data set; these stand in for it):
  * banded LCP batches: symmetric band matrices with off-diagonals U(-1, 1)
    and diagonal = sum of |off-diagonals| + U(0.5, 1.5); right-hand side
    N(mean, 1); sizes uniform in [nmin, nmax];
  * one long band system for the partitioned solve: off-diagonals
    U(-1, 1) drawn independently above and below (not symmetric), diagonal
    as above, right-hand side N(mean, 1);
  * EHL line-contact sweeps: Moes M log-uniform, L uniform;
  * roughness: a sinusoid of given amplitude and wavelength.
"""
import numpy as np

WL_LCP = 2
WL_EHL_SWEEP = 3
WL_EHL_ADJOINT = 4
WL_LONG = 5


def lcp_sizes(count, nmin=513, nmax=4097, seed=0):
    rng = np.random.default_rng([WL_LCP, seed, 1 << 30])
    return rng.integers(nmin, nmax + 1, size=count).astype(np.int64)


def lcp_system(n, q, seed=0, item=0, rhs_mean=0.0):
    """One symmetric, strictly diagonally dominant band system.

    Returns (band, f): band has shape (n, 2q+1) with band[i, d] = a(i, i+d-q);
    entries whose column is outside [0, n) are 0."""
    rng = np.random.default_rng([WL_LCP, seed, item, q])
    n = int(n)
    band = np.zeros((n, 2 * q + 1))
    if n == 0:
        return band, np.zeros(0)
    up = rng.uniform(-1.0, 1.0, size=(n, q))          # a(i, i+d), d = 1..q
    for d in range(1, q + 1):
        up[max(n - d, 0):, d - 1] = 0.0               # column outside the matrix
        band[:, q + d] = up[:, d - 1]
        if d < n:
            band[d:, q - d] = up[: n - d, d - 1]      # a(i, i-d) = a(i-d, i)
    off = np.abs(band).sum(axis=1)
    band[:, q] = off + rng.uniform(0.5, 1.5, size=n)
    f = rng.normal(rhs_mean, 1.0, size=n)
    return band, f


def long_system(n, q, seed=0, rhs_mean=0.0):
    """One non-symmetric, strictly diagonally dominant band system of order n
    (same layout as lcp_system)."""
    rng = np.random.default_rng([WL_LONG, seed, q])
    n = int(n)
    band = rng.uniform(-1.0, 1.0, size=(n, 2 * q + 1))
    cols = np.arange(n)[:, None] + np.arange(-q, q + 1)[None, :]
    band[(cols < 0) | (cols >= n)] = 0.0
    band[:, q] = 0.0
    band[:, q] = np.abs(band).sum(axis=1) + rng.uniform(0.5, 1.5, size=n)
    f = rng.normal(rhs_mean, 1.0, size=n)
    return band, f


def lcp_batch(count, q, nmin=513, nmax=4097, seed=0, rhs_mean=0.0, sizes=None):
    """Batch of band systems concatenated by row offsets.

    Returns (offsets[count+1] int64, band[total, 2q+1], f[total])."""
    if sizes is None:
        sizes = lcp_sizes(count, nmin, nmax, seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    total = int(offsets[-1])
    band = np.empty((total, 2 * q + 1))
    f = np.empty(total)
    for s, n in enumerate(sizes):
        b_s, f_s = lcp_system(int(n), q, seed, s, rhs_mean)
        band[offsets[s]:offsets[s + 1]] = b_s
        f[offsets[s]:offsets[s + 1]] = f_s
    return offsets, band, f


def ehl_sweep_params(count, seed=0, mlo=10.0, mhi=1000.0, llo=5.0, lhi=20.0):
    """Moes parameters for a line-contact sweep: M log-uniform, L uniform."""
    rng = np.random.default_rng([WL_EHL_SWEEP, seed])
    M = np.exp(rng.uniform(np.log(mlo), np.log(mhi), size=count))
    L = rng.uniform(llo, lhi, size=count)
    return M, L


def ehl_adjoint_params(count, seed=0, mlo=20.0, mhi=500.0, L=10.0):
    rng = np.random.default_rng([WL_EHL_ADJOINT, seed])
    M = np.exp(rng.uniform(np.log(mlo), np.log(mhi), size=count))
    return M, np.full(count, L)


def roughness(x, amplitude=0.1, wavelength=0.25, phase=0.0):
    """Sinusoidal surface-roughness profile sampled on the grid ``x``."""
    return amplitude * np.sin(2.0 * np.pi * np.asarray(x) / wavelength + phase)
