"""Adjoint of the converged line contact on the GPU.

  * at the oracle's own converged state (no value comes from the GPU path),
    the GPU gradients dH0/dM, dH0/dL, dHmin/dM, dHmin/dL and the roughness
    gradients match the oracle's dense adjoint within 1e-7 of the largest
    gradient entry: the Jacobian has a condition number of about 1e9 at
    these sizes, so two solvers that are each backward stable (dense LU;
    GMRES to a relative residual of 1e-12) agree to about cond * 1e-16;
  * GPU gradients against central differences (step 1e-6 relative) of
    re-converged GPU solutions, within 1e-5 relative;
  * the same at the oracle's converged kappa-scheme state (kappa = 1/3);
  * the autograd wrapper and a batch of instances with different M on a
    2049-node grid.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import ehl_adjoint as OA
from oracle import ehl_line as OE

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda")
N = 257
AMP = 0.02  # roughness amplitude at which the Newton iteration converges


CASES = [(20.0, 10.0, AMP), (50.0, 8.0, AMP), (100.0, 12.0, 0.0)]


@pytest.fixture(scope="module")
def oracle_states():
    x, _ = OE.grid(N)
    out = []
    for M, L, amp in CASES:
        rough = synth.roughness(x, amplitude=amp)
        r = OE.solve_line(M, L, N, rough=rough)
        assert r["status"] == 0
        g = OA.adjoint_gradients(r["P"], r["H0"], M, L, N, rough=rough)
        out.append((M, L, r, g, rough))
    return out


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def test_adjoint_matches_oracle_at_oracle_state(gpu, oracle_states):
    """Several problems in a row in one process: the workspace of one call
    is reused (uninitialised) by the next."""
    E = gpu.ehl
    for M, L, r, g, rough in oracle_states:
        P, H0, rg = _t(r["P"][None]), _t([r["H0"]]), _t(rough[None])
        a0 = E.adjoint([M], [L], N, P, H0, gH0=_t([1.0]), rough=rg)
        gH = np.zeros((1, N))
        gH[0, g["argmin"]] = 1.0
        a1 = E.adjoint([M], [L], N, P, H0, gH=_t(gH), rough=rg)
        torch.cuda.synchronize()
        assert int(a0["status"][0]) == 0 and int(a1["status"][0]) == 0
        for a, name in ((a0, "H0"), (a1, "Hmin")):
            dr = a["drough"][0].cpu().numpy()
            ref = g[f"d{name}_drough"]
            assert np.abs(dr - ref).max() <= 1e-7 * np.abs(ref).max(), (M, L, name)
            for p in ("M", "L"):
                v, ref = float(a[f"d{p}"][0]), g[f"d{name}_d{p}"]
                assert abs(v - ref) <= 1e-7 * abs(ref), (M, L, name, p, v, ref)


def test_adjoint_kappa_scheme_matches_oracle(gpu):
    """kappa-scheme convection (kappa = 1/3): GPU gradients at the oracle's
    converged kappa-scheme state against the oracle's dense adjoint."""
    E = gpu.ehl
    k, M, L = 1.0 / 3.0, 20.0, 10.0
    r = OE.solve_line(M, L, N, kappa=k)
    assert r["status"] == 0
    g = OA.adjoint_gradients(r["P"], r["H0"], M, L, N, kappa=k)
    opts = E.default_opts(convection=1, kappa=k)
    P, H0 = _t(r["P"][None]), _t([r["H0"]])
    a0 = E.adjoint([M], [L], N, P, H0, gH0=_t([1.0]), opts=opts)
    gH = np.zeros((1, N))
    gH[0, g["argmin"]] = 1.0
    a1 = E.adjoint([M], [L], N, P, H0, gH=_t(gH), opts=opts)
    torch.cuda.synchronize()
    assert int(a0["status"][0]) == 0 and int(a1["status"][0]) == 0
    for a, name in ((a0, "H0"), (a1, "Hmin")):
        dr = a["drough"][0].cpu().numpy()
        ref = g[f"d{name}_drough"]
        assert np.abs(dr - ref).max() <= 1e-7 * np.abs(ref).max(), name
        for p in ("M", "L"):
            v, ref = float(a[f"d{p}"][0]), g[f"d{name}_d{p}"]
            assert abs(v - ref) <= 1e-7 * abs(ref), (name, p, v, ref)


def _solve(E, M, L, rough=None):
    r = E.solve_line(M, L, N, rough=rough)
    torch.cuda.synchronize()
    assert (r["status"] == 0).all()
    return r


def test_adjoint_vs_central_differences(gpu):
    E = gpu.ehl
    x, _ = OE.grid(N)
    rg = _t(synth.roughness(x, amplitude=AMP)[None])
    M, L, step = 50.0, 8.0, 1e-6
    r = _solve(E, [M], [L], rg)
    m = int(torch.argmin(r["H"][0]))
    gH = torch.zeros(1, N, dtype=torch.float64, device=DEV)
    gH[0, m] = 1.0
    aH0 = E.adjoint([M], [L], N, r["P"], r["H0"], gH0=_t([1.0]), rough=rg)
    aHm = E.adjoint([M], [L], N, r["P"], r["H0"], gH=gH, rough=rg)
    torch.cuda.synchronize()
    assert int(aH0["status"][0]) == 0 and int(aHm["status"][0]) == 0
    rp, rm = _solve(E, [M * (1 + step)], [L], rg), _solve(E, [M * (1 - step)], [L], rg)
    fd = (float(rp["H0"][0]) - float(rm["H0"][0])) / (2 * step * M)
    assert abs(fd - float(aH0["dM"][0])) <= 1e-5 * abs(fd)
    rp, rm = _solve(E, [M], [L * (1 + step)], rg), _solve(E, [M], [L * (1 - step)], rg)
    assert int(torch.argmin(rp["H"][0])) == int(torch.argmin(rm["H"][0])) == m
    fd = (float(rp["Hmin"][0]) - float(rm["Hmin"][0])) / (2 * step * L)
    assert abs(fd - float(aHm["dL"][0])) <= 1e-5 * abs(fd)
    for node in (m, m - 7, 120):
        e = torch.zeros_like(rg)
        e[0, node] = step
        rp, rm = _solve(E, [M], [L], rg + e), _solve(E, [M], [L], rg - e)
        fd = (float(rp["Hmin"][0]) - float(rm["Hmin"][0])) / (2 * step)
        v = float(aHm["drough"][0, node])
        assert abs(fd - v) <= 1e-5 * max(1.0, abs(fd)), (node, fd, v)


def test_autograd_function(gpu):
    E = gpu.ehl
    x, _ = OE.grid(N)
    Ms = torch.tensor([20.0, 40.0, 60.0], dtype=torch.float64, requires_grad=True)
    Ls = torch.tensor([10.0, 10.0, 10.0], dtype=torch.float64, requires_grad=True)
    rough = _t(np.stack([synth.roughness(x, amplitude=a) for a in (AMP, AMP, 0.01)]))
    rough.requires_grad_(True)
    P, H0, H, status = E.LineEHL.apply(Ms, Ls, rough, N)
    assert (status == 0).all()
    loss = H.min(dim=1).values.sum() + 0.5 * H0.sum()
    loss.backward()
    m = torch.argmin(H.detach(), dim=1)
    gH = torch.zeros_like(H.detach())
    gH[torch.arange(3), m] = 1.0
    a = E.adjoint(Ms.detach(), Ls.detach(), N, P.detach(), H0.detach(),
                  gH0=torch.full((3,), 0.5, dtype=torch.float64, device=DEV), gH=gH,
                  rough=rough.detach())
    torch.cuda.synchronize()
    assert (a["status"] == 0).all()
    assert torch.allclose(Ms.grad, a["dM"].cpu(), rtol=1e-12, atol=0)
    assert torch.allclose(Ls.grad, a["dL"].cpu(), rtol=1e-12, atol=0)
    assert torch.allclose(rough.grad, a["drough"], rtol=1e-12, atol=0)


def test_batch_2049_gradients_finite_and_fd(gpu):
    """The first instances of the adjoint batch on the 2049-node grid (M
    log-uniform in [20, 500], L = 10, roughness 0.005 sin(2 pi X / 0.25)):
    every instance converges, every gradient is finite, and dH0/dM of two
    instances matches central differences of re-converged solutions."""
    E = gpu.ehl
    NN = 2049
    x, _ = OE.grid(NN)
    Ms, Ls = synth.ehl_adjoint_params(64, seed=0)
    Ms, Ls = Ms[:6], Ls[:6]
    rg = _t(np.stack([synth.roughness(x, amplitude=0.005)] * 6))
    r = E.solve_line(Ms, Ls, NN, rough=rg)
    torch.cuda.synchronize()
    ok = (r["status"] == 0).cpu().numpy()
    assert ok.all(), r["status"].tolist()
    a = E.adjoint(Ms, Ls, NN, r["P"], r["H0"], gH0=torch.ones(6, dtype=torch.float64, device=DEV),
                  rough=rg)
    torch.cuda.synchronize()
    st = a["status"].cpu().numpy()
    assert (st == 0).all(), st.tolist()
    assert torch.isfinite(a["drough"]).all()
    step = 1e-6
    for b in (0, 1):
        Mp, Mm = Ms.copy(), Ms.copy()
        Mp[b] *= 1 + step
        Mm[b] *= 1 - step
        rp = E.solve_line(Mp[b:b + 1], Ls[b:b + 1], NN, rough=rg[b:b + 1].contiguous())
        rm = E.solve_line(Mm[b:b + 1], Ls[b:b + 1], NN, rough=rg[b:b + 1].contiguous())
        torch.cuda.synchronize()
        assert int(rp["status"][0]) == 0 and int(rm["status"][0]) == 0
        fd = (float(rp["H0"][0]) - float(rm["H0"][0])) / (2 * step * Ms[b])
        assert abs(fd - float(a["dM"][b])) <= 1e-5 * abs(fd), (b, fd, float(a["dM"][b]))


def test_autograd_unconverged_forward_gives_nan(gpu):
    """The adjoint is the derivative of a converged fixed point: an instance
    whose forward solve stopped early gets NaN gradients, a converged one in
    the same batch its adjoint gradients."""
    E = gpu.ehl
    Ms = torch.tensor([20.0, 20.0], dtype=torch.float64, requires_grad=True)
    Ls = torch.tensor([10.0, 10.0], dtype=torch.float64, requires_grad=True)
    opts = E.default_opts(max_newton=3, steps_per_graph=1)
    P, H0, H, st = E.LineEHL.apply(Ms, Ls, None, N, opts)
    assert st.cpu().tolist() == [6, 6]
    H0.sum().backward()
    assert torch.isnan(Ms.grad).all() and torch.isnan(Ls.grad).all()
    # converged: finite gradients equal to the adjoint's
    Ms2 = torch.tensor([20.0], dtype=torch.float64, requires_grad=True)
    Ls2 = torch.tensor([10.0], dtype=torch.float64, requires_grad=True)
    P2, H02, H2, st2 = E.LineEHL.apply(Ms2, Ls2, None, N, None)
    assert int(st2[0]) == 0
    H02.sum().backward()
    assert torch.isfinite(Ms2.grad).all() and torch.isfinite(Ls2.grad).all()


def test_adjoint_invalid_arguments(gpu):
    E = gpu.ehl
    P = torch.zeros(1, N, dtype=torch.float64, device=DEV)
    H0 = torch.zeros(1, dtype=torch.float64, device=DEV)
    with pytest.raises(RuntimeError):
        E.adjoint([20.0], [10.0], N, P, H0, rtol=0.0)
    with pytest.raises(RuntimeError):
        E.adjoint([20.0], [10.0], N, P, H0, max_iter=0)
