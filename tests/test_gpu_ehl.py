"""EHL kernels on the GPU vs the FP64 oracle.

Tolerances:
  * deformation FP64 (MFMA f64): differs from the oracle's matmul only in the
    summation order, relative error <= 1e-13 of max|H_el|;  FP32 MFMA over K
    terms: 8 sqrt(K) u32 (u32 = 2^-24, random-walk accumulation bound);
    split-BF16 (x = hi + lo, hi*hi + hi*lo + lo*hi, FP32 accumulation): each
    product keeps 16 mantissa bits, so 4 * 3 * 2^-16 ~ 2e-4;
  * assembly (residual, band of -dR/dsigma, right-hand side): FP64 elementwise
    formulas in a different evaluation order (pow/exp of the lubricant model):
    1e-11 of the row scale plus 1e-14 of the instance scale (rows near the
    cavitation boundary are differences of terms as large as the instance
    scale, so their rounding error is absolute); masks exact;
  * the same for the Lhs1 / Lhs2 splitting matrices (eqs. 60-61) and the
    fixed point those iterations reach;
  * converged Newton solution: P, H, H0, Hmin within 1e-10 relative (the
    stated FP64 target); both sides iterate to max|dP| <= 1e-13.
"""
import numpy as np
import pytest
import torch

from oracle import deform as odef
from oracle import ehl_line as OE

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda")


def _rel(a, b):
    return np.abs(a - b).max() / max(1e-300, np.abs(b).max())


U32 = 2.0 ** -24


def _tol(prec, K):
    return {0: 1e-13, 3: 8 * np.sqrt(K) * U32, 2: 2e-4}[prec]


@pytest.mark.parametrize("N,B", [(5, 1), (17, 3), (130, 33), (257, 40), (1025, 5), (2049, 33),
                                 (4097, 7), (6001, 2)])
@pytest.mark.parametrize("prec", [0, 3, 2])
def test_line_deformation(gpu, N, B, prec):
    """K P against the oracle's dense product: ragged row and column tiles,
    several P chunks, the workload's N = 4097, and N = 6001, where the FP64
    kernel vector no longer fits the tiled kernel's LDS (untiled kernel)."""
    tol = _tol(prec, N)
    P = gpu.ehl
    x, h = OE.grid(N)
    rng = np.random.default_rng(N + B)
    Pin = np.abs(rng.normal(size=(B, N))) * OE.hertz_start(x)[None, :]
    Pin[:, 0] = Pin[:, -1] = 0.0
    out = P.deformation(torch.as_tensor(Pin, device=DEV), P.line_grid(N), prec=prec)
    ref = odef.line_deformation(Pin.T, h).T
    assert _rel(out.cpu().numpy(), ref) < tol


@pytest.mark.parametrize("Nx,Ny,B", [(9, 7, 1), (33, 33, 2), (65, 65, 1), (129, 97, 1),
                                     (17, 130, 3), (40, 257, 1), (70, 64, 2)])
@pytest.mark.parametrize("prec", [0, 3, 2])
def test_point_deformation(gpu, Nx, Ny, B, prec):
    """H_el = K P of point grids against the oracle's direct sum: ragged
    tiles and chunks along y (Ny = 7, 97, 130, 257), along x (Nx = 17, 70)
    and several instances."""
    tol = _tol(prec, Nx * Ny)
    P = gpu.ehl
    grid = P.point_grid(Nx, Ny)
    hx = (grid.x1 - grid.x0) / (Nx - 1)
    hy = (grid.y1 - grid.y0) / (Ny - 1)
    rng = np.random.default_rng(Nx * Ny)
    Pin = rng.random((B, Nx, Ny))
    out = P.deformation(torch.as_tensor(Pin, device=DEV), grid, prec=prec).cpu().numpy()
    for b in range(B):
        ref = odef.point_deformation(Pin[b], hx, hy)
        assert _rel(out[b], ref) < tol


def _state(N, seed):
    x, h = OE.grid(N)
    kvec = odef.line_kernel(N, h)
    rng = np.random.default_rng(seed)
    P = OE.hertz_start(x) * (1 + 0.2 * rng.random(N))
    P[0] = P[-1] = 0.0
    P[int(0.8 * N):int(0.8 * N) + 4] = 0.0
    return x, h, kvec, P


@pytest.mark.parametrize("N", [9, 65, 257, 700])
@pytest.mark.parametrize("kterms", [1, 2])
@pytest.mark.parametrize("limjac", [0, 1, 2])
def test_line_assembly(gpu, N, kterms, limjac):
    P = gpu.ehl
    Ms, Ls, H0s = [20.0, 100.0, 500.0], [10.0, 5.0, 20.0], [-0.3, -0.55, -0.58]
    x, h, kvec, _ = _state(N, 0)
    Ps = np.stack([_state(N, s)[3] for s in range(3)])
    rough = 0.01 * np.sin(2 * np.pi * x / 0.25)[None, :].repeat(3, 0)
    Hel = np.stack([odef.line_deformation(Ps[b], h) for b in range(3)])
    opts = P.default_opts(kernel_terms=kterms, limiter_jacobian=limjac)
    r = P.assemble(P.line_grid(N), P.params_tensor(Ms, Ls, DEV), torch.as_tensor(Ps, device=DEV),
                   torch.as_tensor(Hel, device=DEV),
                   torch.as_tensor(H0s, dtype=torch.float64, device=DEV), opts,
                   rough=torch.as_tensor(rough, device=DEV))
    g = {k: v.cpu().numpy() for k, v in r.items()}
    for b in range(3):
        _, lam, ph = OE.moes_line(Ms[b], Ls[b])
        H = H0s[b] + 0.5 * x * x + Hel[b] + rough[b]
        R, st = OE.residual(Ps[b], H, ph, lam, h)
        direct_all = OE.hybrid_direct(Ps[b], st["eps"], h)
        direct = direct_all[1:-1]
        A = -OE.jacobian_band(Ps[b], H, ph, lam, h, kvec, direct, kterms, limjac)
        rhs = OE.band_matvec(A, Ps[b][1:-1]) + R
        nb = np.concatenate([[True], direct, [True]])
        bounded = (direct & nb[:-2] & nb[2:]).astype(np.uint8)
        assert (g["direct"][b] == direct_all.astype(np.uint8)).all()
        assert (g["bounded"][b] == bounded).all()
        scale = np.abs(A).max(axis=1, keepdims=True)
        assert (np.abs(g["band"][b] - A) <= 1e-11 * scale + 1e-14 * np.abs(A).max()).all()
        assert _rel(g["R"][b], R) < 1e-11
        assert np.abs(g["rhs"][b] - rhs).max() <= 1e-11 * max(1, np.abs(rhs).max())


@pytest.mark.parametrize("N", [65, 700])
@pytest.mark.parametrize("split,kappa", [(1, None), (2, None), (1, 1.0 / 3.0), (2, -1.0)])
def test_line_assembly_splitting(gpu, N, split, kappa):
    """The Lhs1 / Lhs2 matrices (eps and rho frozen, upwind convective
    derivative weighted by (2-k)/2 or (2-k)/2 + (1-k)/4) and the right-hand
    side built on them, against the oracle."""
    P = gpu.ehl
    Ms, Ls, H0s = [20.0, 100.0, 500.0], [10.0, 5.0, 20.0], [-0.3, -0.55, -0.58]
    x, h, kvec, _ = _state(N, 0)
    Ps = np.stack([_state(N, s)[3] for s in range(3)])
    Hel = np.stack([odef.line_deformation(Ps[b], h) for b in range(3)])
    opts = P.default_opts(kernel_terms=2, convection=0 if kappa is None else 1,
                          kappa=0.0 if kappa is None else kappa, splitting=split)
    r = P.assemble(P.line_grid(N), P.params_tensor(Ms, Ls, DEV), torch.as_tensor(Ps, device=DEV),
                   torch.as_tensor(Hel, device=DEV),
                   torch.as_tensor(H0s, dtype=torch.float64, device=DEV), opts)
    g = {k: v.cpu().numpy() for k, v in r.items()}
    for b in range(3):
        _, lam, ph = OE.moes_line(Ms[b], Ls[b])
        H = H0s[b] + 0.5 * x * x + Hel[b]
        R, st = OE.residual(Ps[b], H, ph, lam, h, kappa)
        direct = OE.hybrid_direct(Ps[b], st["eps"], h)[1:-1]
        A = -OE.jacobian_band(Ps[b], H, ph, lam, h, kvec, direct, 2, kappa=kappa, split=split)
        rhs = OE.band_matvec(A, Ps[b][1:-1]) + R
        scale = np.abs(A).max(axis=1, keepdims=True)
        assert (np.abs(g["band"][b] - A) <= 1e-11 * scale + 1e-14 * np.abs(A).max()).all()
        assert _rel(g["R"][b], R) < 1e-11
        assert np.abs(g["rhs"][b] - rhs).max() <= 1e-11 * max(1, np.abs(rhs).max())


@pytest.mark.parametrize("split,kappa", [(1, None), (2, None), (2, 1.0 / 3.0)])
def test_newton_splitting_matches_oracle(gpu, split, kappa):
    """Config 1 iterated with the Lhs1 / Lhs2 matrices (eqs. 60-61) instead
    of the Newton band: the GPU and the oracle, run the same way, agree on the
    fixed point within 1e-10."""
    o = OE.solve_line(20.0, 10.0, 257, kappa=kappa, splitting=split)
    assert o["status"] == 0
    P = gpu.ehl
    r = P.solve_line([20.0], [10.0], 257,
                     opts=P.default_opts(convection=0 if kappa is None else 1,
                                         kappa=0.0 if kappa is None else kappa,
                                         splitting=split))
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 0
    assert _rel(r["P"][0].cpu().numpy(), o["P"]) < 1e-10
    assert abs(float(r["H0"][0]) - o["H0"]) <= 1e-10 * abs(o["H0"])
    assert abs(float(r["Hmin"][0]) - o["Hmin"]) <= 1e-10 * abs(o["Hmin"])
    assert abs(int(r["iters"][0]) - o["iters"]) <= 5


@pytest.fixture(scope="module")
def oracle_cfg1():
    r = OE.solve_line(20.0, 10.0, 257)
    assert r["status"] == 0
    return r


def test_newton_config1_matches_oracle(gpu, oracle_cfg1):
    """Config 1: one instance, N=257, M=20, L=10, Hertzian start."""
    P = gpu.ehl
    o = oracle_cfg1
    r = P.solve_line([20.0], [10.0], 257)
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 0
    Pg = r["P"][0].cpu().numpy()
    assert _rel(Pg, o["P"]) < 1e-10
    assert _rel(r["H"][0].cpu().numpy(), o["H"]) < 1e-10
    assert abs(float(r["H0"][0]) - o["H0"]) <= 1e-10 * abs(o["H0"])
    assert abs(float(r["Hmin"][0]) - o["Hmin"]) <= 1e-10 * abs(o["Hmin"])
    assert abs(int(r["iters"][0]) - o["iters"]) <= 5


def test_newton_batch_matches_oracle(gpu):
    """Several instances of a sweep in one batched call (N=257)."""
    P = gpu.ehl
    Ms = [10.0, 20.0, 50.0, 100.0]
    Ls = [5.0, 10.0, 15.0, 10.0]
    r = P.solve_line(Ms, Ls, 257)
    torch.cuda.synchronize()
    st = r["status"].cpu().numpy()
    for b, (M, L) in enumerate(zip(Ms, Ls)):
        o = OE.solve_line(M, L, 257)
        assert o["status"] == st[b] == 0, (M, L, o["status"], st[b])
        assert _rel(r["P"][b].cpu().numpy(), o["P"]) < 1e-10
        assert abs(float(r["H0"][b]) - o["H0"]) <= 1e-10 * abs(o["H0"])
        assert abs(float(r["Hmin"][b]) - o["Hmin"]) <= 1e-10 * abs(o["Hmin"])


def test_newton_mixed_deformation_refreshed(gpu, oracle_cfg1):
    """FP32 / split-BF16 deformation with a final FP64 phase reaches the same
    fixed point within 1e-8 (the mixed-path target)."""
    P = gpu.ehl
    o = oracle_cfg1
    for prec in (3, 2):
        r = P.solve_line([20.0], [10.0], 257, opts=P.default_opts(deform_prec=prec))
        torch.cuda.synchronize()
        assert int(r["status"][0]) == 0
        assert _rel(r["P"][0].cpu().numpy(), o["P"]) < 1e-8
        assert abs(float(r["Hmin"][0]) - o["Hmin"]) <= 1e-8 * abs(o["Hmin"])


def test_newton_fp32_refined_lcp_matches_oracle(gpu, oracle_cfg1):
    """lcp_prec = FP32 factors + FP64 refinement inside every Newton step:
    the same fixed point within the mixed-path target 1e-8."""
    P = gpu.ehl
    o = oracle_cfg1
    r = P.solve_line([20.0], [10.0], 257, opts=P.default_opts(lcp_prec=P.B.PREC_FP32_IR))
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 0
    assert _rel(r["P"][0].cpu().numpy(), o["P"]) < 1e-8
    assert _rel(r["H"][0].cpu().numpy(), o["H"]) < 1e-8
    assert abs(float(r["H0"][0]) - o["H0"]) <= 1e-8 * abs(o["H0"])
    assert abs(float(r["Hmin"][0]) - o["Hmin"]) <= 1e-8 * abs(o["Hmin"])


def test_newton_forced_lcp_cap_status(gpu):
    """An active-set cap of one solve fails the first step's LCP on the GPU
    (its first step starts from the empty set, which is not the solution's
    active set); with lcp_fail_steps = 1 the instance stops there with
    SYS_LCP_NOT_CONVERGED.  The oracle (sign-of-b start, whose first step
    happens to need one solve) stops with the same status a step later."""
    P = gpu.ehl
    o = OE.solve_line(20.0, 10.0, 129, lcp_max_iter=1, lcp_fail_steps=1)
    r = P.solve_line([20.0, 20.0], [10.0, 10.0], 129,
                     opts=P.default_opts(lcp_max_iter=1, lcp_fail_steps=1, steps_per_graph=1))
    torch.cuda.synchronize()
    assert o["status"] == 3 and o["iters"] <= 3
    assert r["status"].cpu().tolist() == [3, 3]
    assert r["iters"].cpu().tolist() == [1, 1]


def test_newton_not_converged_status(gpu):
    P = gpu.ehl
    r = P.solve_line([20.0], [10.0], 257, opts=P.default_opts(max_newton=3, steps_per_graph=1))
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 6
    assert int(r["iters"][0]) == 3


KAPPA_CASES = [0.0, 1.0 / 3.0, -1.0]


@pytest.mark.parametrize("N", [65, 700])
@pytest.mark.parametrize("limjac", [0, 2])
@pytest.mark.parametrize("kappa", KAPPA_CASES)
def test_line_assembly_kappa_scheme(gpu, N, limjac, kappa):
    """kappa-scheme convection (Sec. 3.3, eqs. 56-59): band, residual, rhs and masks of the
    GPU assembly against the oracle's, same bounds as the van Leer case."""
    P = gpu.ehl
    Ms, Ls, H0s = [20.0, 100.0], [10.0, 5.0], [-0.3, -0.55]
    x, h, kvec, _ = _state(N, 0)
    Ps = np.stack([_state(N, s)[3] for s in range(2)])
    Hel = np.stack([odef.line_deformation(Ps[b], h) for b in range(2)])
    opts = P.default_opts(kernel_terms=2, limiter_jacobian=limjac, convection=1, kappa=kappa)
    r = P.assemble(P.line_grid(N), P.params_tensor(Ms, Ls, DEV), torch.as_tensor(Ps, device=DEV),
                   torch.as_tensor(Hel, device=DEV),
                   torch.as_tensor(H0s, dtype=torch.float64, device=DEV), opts)
    g = {k: v.cpu().numpy() for k, v in r.items()}
    for b in range(2):
        _, lam, ph = OE.moes_line(Ms[b], Ls[b])
        H = H0s[b] + 0.5 * x * x + Hel[b]
        R, st = OE.residual(Ps[b], H, ph, lam, h, kappa)
        direct = OE.hybrid_direct(Ps[b], st["eps"], h)[1:-1]
        A = -OE.jacobian_band(Ps[b], H, ph, lam, h, kvec, direct, 2, limjac, kappa)
        rhs = OE.band_matvec(A, Ps[b][1:-1]) + R
        scale = np.abs(A).max(axis=1, keepdims=True)
        assert (np.abs(g["band"][b] - A) <= 1e-11 * scale + 1e-14 * np.abs(A).max()).all()
        assert _rel(g["R"][b], R) < 1e-11
        assert np.abs(g["rhs"][b] - rhs).max() <= 1e-11 * max(1, np.abs(rhs).max())


@pytest.mark.parametrize("kappa", KAPPA_CASES)
def test_newton_config1_kappa_scheme_matches_oracle(gpu, kappa):
    P = gpu.ehl
    o = OE.solve_line(20.0, 10.0, 257, kappa=kappa)
    assert o["status"] == 0
    r = P.solve_line([20.0], [10.0], 257, opts=P.default_opts(convection=1, kappa=kappa))
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 0
    assert _rel(r["P"][0].cpu().numpy(), o["P"]) < 1e-10
    assert abs(float(r["H0"][0]) - o["H0"]) <= 1e-10 * abs(o["H0"])
    assert abs(float(r["Hmin"][0]) - o["Hmin"]) <= 1e-10 * abs(o["Hmin"])


def test_kappa_scheme_rejected_where_not_supported(gpu):
    P = gpu.ehl
    # the library refuses the options (the workspace query returns 0 for
    # invalid options, the solve returns PAQIF_EINVAL)
    with pytest.raises((RuntimeError, ValueError)):  # out of range
        P.solve_line([20.0], [10.0], 65, opts=P.default_opts(convection=1, kappa=1.5))
