"""Convection-diffusion workload on the GPU vs the FP64 oracle.

  * the example set-up (f for x^4 + y^4, start iterate) elementwise (1e-14);
  * the line relaxation after a fixed number of iterations: the iterate
    within 1e-10 of the oracle's (same half-steps; the line solves differ in
    method -- PAQIF without pivoting vs banded LU with partial pivoting --
    and summation order, which the well-conditioned line systems keep at a
    few ulps per step); n = 13 (one PAQIF superblock per line), 34 (even
    line order) and 65 (several superblocks, ragged last one);
  * at convergence (max defect <= 1e-12 max|f|): the same iteration count
    within one and the same discrete solution within 1e-10;
  * the distributive line relaxation (Ls3): the iterate after a fixed number
    of iterations within 1e-10 of the oracle's (n = 13, 34), and on 9 x 9
    nodes the converged solution within 1e-10 with the iteration count
    within one;
  * the x-line splittings Ls0 / Ls1 (two colours per sweep): the iterate
    after a fixed number of sweeps within 1e-10 of the oracle's (n = 13, 34,
    65), and on 33 x 33 nodes the converged solution within 1e-10 with the
    sweep count within one;
  * argument checks.
"""
import numpy as np
import pytest
import torch

from oracle import convdiff as C

pytestmark = pytest.mark.gpu
KAPPAS = [0.0, 1.0 / 3.0, -1.0]


def test_example_setup(gpu):
    n, eps = 33, 1e-6
    f, u = gpu.convdiff.example(n, eps)
    assert np.abs(f.cpu().numpy() - C.rhs(n, eps)).max() <= 1e-14 * np.abs(C.rhs(n, eps)).max()
    assert np.abs(u.cpu().numpy() - C.start(n)).max() <= 1e-14 * 2


def _oracle_iterate(n, kappa, eps, omega, iters):
    f = C.rhs(n, eps)
    u = C.start(n)
    for _ in range(iters):
        u = C.half_step(u, f, 0, kappa, eps, omega)
        u = C.half_step(u, f, 1, kappa, eps, omega)
    return u


@pytest.mark.parametrize("n", [13, 34, 65])
@pytest.mark.parametrize("kappa", KAPPAS)
def test_fixed_iterations_match_oracle(gpu, n, kappa):
    eps, omega, k = 1e-6, 0.9, 6
    f, u = gpu.convdiff.example(n, eps)
    it, _ = gpu.convdiff.line_relax(f, u, kappa, eps, omega=omega, tol=0.0, max_iter=k)
    torch.cuda.synchronize()
    assert it == k
    ref = _oracle_iterate(n, kappa, eps, omega, k)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("kappa", KAPPAS)
def test_converged_solution_matches_oracle(gpu, kappa):
    n, eps = 33, 1e-6
    o = C.solve(n, kappa, eps=eps, tol=1e-12, max_iter=400)
    f, u = gpu.convdiff.example(n, eps)
    it, res = gpu.convdiff.line_relax(f, u, kappa, eps, tol=1e-12, max_iter=400)
    torch.cuda.synchronize()
    assert res <= 1e-12 * o["fmax"]
    assert abs(it - o["iters"]) <= 1
    assert np.abs(u.cpu().numpy() - o["u"]).max() <= 1e-10 * np.abs(o["u"]).max()


def test_invalid_arguments(gpu):
    f, u = gpu.convdiff.example(17)
    for kw in (dict(kappa=1.0), dict(kappa=0.0, omega=0.0), dict(kappa=0.0, a=-1.0),
               dict(kappa=0.0, max_iter=0)):
        with pytest.raises(RuntimeError):
            gpu.convdiff.line_relax(f, u, **kw)
    with pytest.raises(RuntimeError):
        gpu.convdiff.example(4)


@pytest.mark.parametrize("n", [13, 34])
@pytest.mark.parametrize("kappa", KAPPAS)
def test_ls3_fixed_iterations_match_oracle(gpu, n, kappa):
    eps, omega, k = 1e-6, 0.9, 4
    f, u = gpu.convdiff.example(n, eps)
    it, _ = gpu.convdiff.distributive_relax(f, u, kappa, eps, omega=omega, tol=0.0, max_iter=k)
    torch.cuda.synchronize()
    assert it == k
    ref = C.start(n)
    fr = C.rhs(n, eps)
    for _ in range(k):
        ref = C.ls3_iteration(ref, fr, kappa, eps, omega)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("kappa", KAPPAS)
def test_ls3_converged_matches_oracle(gpu, kappa):
    n = 9
    o = C.solve_ls3(n, kappa, tol=1e-11, max_iter=600)
    f, u = gpu.convdiff.example(n, 1e-6)
    it, res = gpu.convdiff.distributive_relax(f, u, kappa, tol=1e-11, max_iter=600)
    torch.cuda.synchronize()
    assert res <= 1e-11 * o["fmax"]
    assert abs(it - o["iters"]) <= 1
    assert np.abs(u.cpu().numpy() - o["u"]).max() <= 1e-10 * np.abs(o["u"]).max()


@pytest.mark.parametrize("n", [13, 34, 65])
@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("kappa", KAPPAS)
def test_split_fixed_iterations_match_oracle(gpu, n, which, kappa):
    eps, omega, k = 1e-6, 0.7, 5
    f, u = gpu.convdiff.example(n, eps)
    it, _ = gpu.convdiff.split_relax(f, u, which, kappa, eps, omega=omega, tol=0.0, max_iter=k)
    torch.cuda.synchronize()
    assert it == k
    ref = C.start(n)
    fr = C.rhs(n, eps)
    for _ in range(k):
        ref = C.split_iteration(ref, fr, which, kappa, eps, omega)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("kappa", KAPPAS)
def test_split_converged_matches_oracle(gpu, which, kappa):
    n = 33
    o = C.solve_split(n, which, kappa, omega=0.7, tol=1e-12, max_iter=2000)
    assert o["defect"] <= 1e-12 * o["fmax"]
    f, u = gpu.convdiff.example(n, 1e-6)
    it, res = gpu.convdiff.split_relax(f, u, which, kappa, omega=0.7, tol=1e-12, max_iter=2000)
    torch.cuda.synchronize()
    assert res <= 1e-12 * o["fmax"]
    assert abs(it - o["iters"]) <= 1
    assert np.abs(u.cpu().numpy() - o["u"]).max() <= 1e-10 * np.abs(o["u"]).max()


def test_split_invalid_arguments(gpu):
    f, u = gpu.convdiff.example(17)
    with pytest.raises(RuntimeError):
        gpu.convdiff.split_relax(f, u, 2, 0.0)
    with pytest.raises(RuntimeError):
        gpu.convdiff.split_relax(f, u, 0, 1.0)
