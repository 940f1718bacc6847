"""EHL point contact on the GPU vs the FP64 oracle.

  * sweep assembly (both directions, both colours): band, rhs and masks of
    every line against the oracle's sweep systems, FP64 elementwise formulas
    in another evaluation order: 1e-11 of the row scale plus 1e-14 of the
    instance scale (the line-contact assembly bound), masks exact;
  * the same with the kappa-scheme convection (kappa = 0, 1/3, -1; exact and
    first-order Newton matrix), and with the Lhs1 / Lhs2 splitting matrices;
  * converged alternating-sweep solution on 33 x 33 nodes (van Leer, and
    the kappa-scheme with kappa = 1/3): P, H0, Hmin within 1e-10 relative
    (both sides stop at max |dP| <= 1e-12 per step; with a contraction of
    about 0.97 per step each is within ~3e-11 of the fixed point: the
    oracle's solution at this stop differs from its solution at 1e-13 by
    6e-12 relative); the Lhs2 splitting reaches the same fixed point;
  * the 257 x 257 contact (M = 200, L = 10): converged, load balance, y-mirror
    symmetry and complementarity of the oracle's residual on the GPU
    solution.
"""
import numpy as np
import pytest
import torch

from oracle import deform as odef
from oracle import ehl_line as OL
from oracle import ehl_point as OP

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda")


def _state(Nx, Ny, seed):
    X, Y, hx, hy = OP.grid(Nx, Ny)
    rng = np.random.default_rng(seed)
    P = OP.hertz_start(X, Y) * (1 + 0.2 * rng.random((Nx, Ny)))
    P[0, :] = P[-1, :] = P[:, 0] = P[:, -1] = 0.0
    P[int(0.75 * Nx):int(0.75 * Nx) + 2, Ny // 3:Ny // 2] = 0.0   # a cavitated patch
    return X, Y, hx, hy, P


@pytest.mark.parametrize("Nx,Ny", [(17, 13), (33, 33)])
@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("kterms", [1, 2])
@pytest.mark.parametrize("limjac", [0, 1])
def test_point_sweep_assembly(gpu, Nx, Ny, axis, kterms, limjac):
    _check_assembly(gpu, Nx, Ny, axis, kterms, limjac, None)


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("limjac", [0, 2])
@pytest.mark.parametrize("kappa", [0.0, 1.0 / 3.0, -1.0])
def test_point_sweep_assembly_kappa_scheme(gpu, axis, limjac, kappa):
    _check_assembly(gpu, 17, 13, axis, 2, limjac, kappa)


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("split,kappa", [(1, None), (2, None), (2, 1.0 / 3.0), (1, -1.0)])
def test_point_sweep_assembly_splitting(gpu, axis, split, kappa):
    """Lhs1 / Lhs2 line matrices (eps and rho frozen, weighted upwind
    convective derivative) and their right-hand sides."""
    _check_assembly(gpu, 17, 13, axis, 2, 2, kappa, split)


def _check_assembly(gpu, Nx, Ny, axis, kterms, limjac, kappa, split=0):
    E = gpu.ehl
    Ms, Ls, H0s = [20.0, 200.0], [10.0, 8.0], [-0.5, -0.9]
    X, Y, hx, hy, _ = _state(Nx, Ny, 0)
    Ps = np.stack([_state(Nx, Ny, s)[4] for s in (1, 2)])
    Hel = np.stack([odef.point_deformation(Ps[b], hx, hy) for b in range(2)])
    k2 = odef.point_kernel(Nx, Ny, hx, hy)
    opts = E.default_opts(kernel_terms=kterms, limiter_jacobian=limjac,
                          convection=0 if kappa is None else 1,
                          kappa=0.0 if kappa is None else kappa, splitting=split)
    grid = E.point_grid(Nx, Ny)
    for color in (1, 0):
        g = E.point_sweep_assemble(grid, E.params_tensor(Ms, Ls, DEV), torch.as_tensor(Ps, device=DEV),
                                   torch.as_tensor(Hel, device=DEV),
                                   torch.as_tensor(H0s, dtype=torch.float64, device=DEV), axis,
                                   color, opts)
        g = {k: v.cpu().numpy() for k, v in g.items()}
        nl = Ny if axis == 0 else Nx
        lines = [l for l in range(1, nl - 1) if l % 2 == color]
        for b in range(2):
            _, lam, ph = OP.moes_point(Ms[b], Ls[b])
            H = H0s[b] + 0.5 * X[:, None] ** 2 + 0.5 * Y[None, :] ** 2 + Hel[b]
            st = OL.state(Ps[b], H, ph, lam)
            direct = OP.classify(Ps[b], st["eps"], hx, hy)
            A, rhs, bounded = OP.sweep_systems(Ps[b], H, st, ph, lam, hx, hy, k2, direct, axis,
                                               kterms, limjac, kappa, split)
            assert (g["direct"][b] == direct.astype(np.uint8)).all()
            inst = np.abs(A).max()
            for slot, l in enumerate(lines):
                sys_ = b * len(lines) + slot
                ref = A[l - 1]
                scale = np.abs(ref).max(axis=1, keepdims=True)
                assert (np.abs(g["band"][sys_] - ref) <= 1e-11 * scale + 1e-14 * inst).all(), \
                    (b, color, l)
                assert (g["bounded"][sys_] == bounded[l - 1]).all()
                rs = max(1.0, np.abs(rhs[l - 1]).max())
                assert np.abs(g["rhs"][sys_] - rhs[l - 1]).max() <= 1e-11 * rs + 1e-14 * inst


@pytest.fixture(scope="module")
def oracle_33():
    r = OP.solve_point(20.0, 10.0, 33, 33, tol=1e-12, max_steps=1500)
    assert r["status"] == 0
    return r


def test_point_newton_matches_oracle(gpu, oracle_33):
    E = gpu.ehl
    o = oracle_33
    r = E.solve_point([20.0], [10.0], 33, 33,
                      opts=E.default_opts(tol=1e-12, max_newton=1500, c_h0=0.02))
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 0
    P = r["P"][0].cpu().numpy()
    assert np.abs(P - o["P"]).max() <= 1e-10 * np.abs(o["P"]).max()
    assert abs(float(r["H0"][0]) - o["H0"]) <= 1e-10 * abs(o["H0"])
    assert abs(float(r["Hmin"][0]) - o["Hmin"]) <= 1e-10 * abs(o["Hmin"])


def test_point_newton_kappa_scheme_matches_oracle(gpu):
    k = 1.0 / 3.0
    o = OP.solve_point(20.0, 10.0, 33, 33, tol=1e-12, max_steps=1500, kappa=k)
    assert o["status"] == 0
    E = gpu.ehl
    r = E.solve_point([20.0], [10.0], 33, 33,
                      opts=E.default_opts(tol=1e-12, max_newton=1500, c_h0=0.02, convection=1,
                                          kappa=k))
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 0
    P = r["P"][0].cpu().numpy()
    assert np.abs(P - o["P"]).max() <= 1e-10 * np.abs(o["P"]).max()
    assert abs(float(r["H0"][0]) - o["H0"]) <= 1e-10 * abs(o["H0"])
    assert abs(float(r["Hmin"][0]) - o["Hmin"]) <= 1e-10 * abs(o["Hmin"])


def test_point_lhs2_splitting_matches_oracle(gpu, oracle_33):
    """The Lhs2 splitting (eq. 61) as the sweeps' line matrices: the oracle's
    Lhs2 iteration and the GPU's reach the Newton fixed point within 1e-10."""
    o2 = OP.solve_point(20.0, 10.0, 33, 33, tol=1e-12, max_steps=1500, splitting=2)
    assert o2["status"] == 0
    E = gpu.ehl
    r = E.solve_point([20.0], [10.0], 33, 33,
                      opts=E.default_opts(tol=1e-12, max_newton=1500, c_h0=0.02, splitting=2))
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 0
    P = r["P"][0].cpu().numpy()
    for o in (o2, oracle_33):
        assert np.abs(P - o["P"]).max() <= 1e-10 * np.abs(o["P"]).max()
        assert abs(float(r["H0"][0]) - o["H0"]) <= 1e-10 * abs(o["H0"])
        assert abs(float(r["Hmin"][0]) - o["Hmin"]) <= 1e-10 * abs(o["Hmin"])
    assert abs(int(r["iters"][0]) - o2["iters"]) <= 10


def test_point_newton_fp32_refined_lcp_matches_oracle(gpu, oracle_33):
    """lcp_prec = FP32 factors + FP64 refinement for every line LCP: the
    same fixed point within the mixed-path target 1e-8."""
    E = gpu.ehl
    o = oracle_33
    r = E.solve_point([20.0], [10.0], 33, 33,
                      opts=E.default_opts(tol=1e-12, max_newton=1500, c_h0=0.02,
                                          lcp_prec=E.B.PREC_FP32_IR))
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 0
    P = r["P"][0].cpu().numpy()
    assert np.abs(P - o["P"]).max() <= 1e-8 * np.abs(o["P"]).max()
    assert abs(float(r["H0"][0]) - o["H0"]) <= 1e-8 * abs(o["H0"])
    assert abs(float(r["Hmin"][0]) - o["Hmin"]) <= 1e-8 * abs(o["Hmin"])


def test_point_forced_lcp_cap_status(gpu):
    """Every line LCP of a colour pass reports its status; with an
    active-set cap of one solve the first step's passes fail (the empty start
    set is not the solution's) and, with lcp_fail_steps = 1, every instance
    stops after that step with SYS_LCP_NOT_CONVERGED."""
    E = gpu.ehl
    r = E.solve_point([20.0, 50.0], [10.0, 10.0], 33, 33,
                      opts=E.default_opts(c_h0=0.02, lcp_max_iter=1, lcp_fail_steps=1,
                                          steps_per_graph=1))
    torch.cuda.synchronize()
    assert r["status"].cpu().tolist() == [3, 3]
    assert r["iters"].cpu().tolist() == [1, 1]
    # the default allows 16 consecutive failures: the same cap does not stop
    # the iteration after one step
    r = E.solve_point([20.0], [10.0], 33, 33,
                      opts=E.default_opts(c_h0=0.02, lcp_max_iter=1, max_newton=4,
                                          steps_per_graph=1))
    torch.cuda.synchronize()
    assert int(r["iters"][0]) == 4 and int(r["status"][0]) == 6


def test_point_config5_properties(gpu):
    """257 x 257, M = 200, L = 10: properties of the GPU solution checked with
    the oracle's residual."""
    E = gpu.ehl
    N = 257
    r = E.solve_point([200.0], [10.0], N, N,
                      opts=E.default_opts(tol=1e-10, max_newton=30000, c_h0=0.02))
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 0, (int(r["status"][0]), int(r["iters"][0]))
    P = r["P"][0].cpu().numpy()
    H0 = float(r["H0"][0])
    X, Y, hx, hy = OP.grid(N, N)
    assert abs(hx * hy * P.sum() - OP.LOAD) <= 1e-9
    assert np.abs(P - P[:, ::-1]).max() <= 1e-9 * P.max()
    assert (P >= 0).all()
    _, lam, ph = OP.moes_point(200.0, 10.0)
    H = OP.film(P, H0, X, Y, hx, hy)
    R, st = OP.residual(P, H, ph, lam, hx, hy)
    Pi = P[1:-1, 1:-1]
    scale = np.abs(st["rH"]).max() / hx          # size of the flux term
    press = Pi > 1e-8
    assert np.abs(R[press]).max() <= 1e-6 * scale
    assert (-R[~press] >= -1e-6 * scale).all()
