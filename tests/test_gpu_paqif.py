"""PAQIF on the GPU vs the FP64 oracle (same seeded inputs, element by element).

The exact mode's starting active set (projected Jacobi sweeps, a handle
setting the autotuner tunes) changes only the number of active-set solves:
the tests compare solutions and active sets exactly, solve counts loosely.

Tolerances: the AQIF solution differs from the oracle only by rounding order
(same elimination order, FP64); on these diagonally dominant systems
(condition number below ~50) the relative difference stays below 1e-12.  The
active set is compared exactly.  Mixed precision (FP32 factors + FP64
iterative refinement to |r| <= 1e-10 |b|): u within 1e-9 relative.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

SIZES_RAGGED = [1, 2, 3, 4, 5, 7, 8, 9, 16, 17, 31, 33, 64, 65, 100, 127, 128, 257, 300, 513]


def _run(P, q, sizes, mode, prec=0, seed=0, rhs_mean=0.0, bounded=None, order=None):
    offs, band, f = synth.lcp_batch(len(sizes), q, seed=seed, rhs_mean=rhs_mean, sizes=sizes)
    bt = P.paqif.Batch(offs, q, order=order)
    dev = torch.device("cuda")
    bnd = None if bounded is None else torch.as_tensor(bounded, dtype=torch.uint8, device=dev)
    r = P.paqif.solve_lcp(bt, torch.as_tensor(band, device=dev), torch.as_tensor(f, device=dev),
                          mode=mode, prec=prec, bounded=bnd)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in r.items()}
    o = oracle.lcp_batch(q, offs, band, f, bounded=bounded, mode=mode)
    return offs, g, o


def _relerr(a, b):
    return np.abs(a - b).max() / max(1.0, np.abs(b).max())


@pytest.mark.parametrize("q", [2, 4, 8])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_parity_ragged(gpu, q, mode):
    offs, g, o = _run(gpu, q, SIZES_RAGGED, mode, seed=q * 10 + mode)
    assert (g["status"] == 0).all(), g["status"]
    assert (o["status"] == 0).all()
    if mode != 2:
        # one solve; exact mode: the solution is unique, the number of
        # active-set solves depends on the start set, compared loosely
        assert (g["iters"] == 1).all() and (o["iters"] == 1).all()
    else:
        assert (np.abs(g["iters"] - o["iters"]) <= 2).all()
    assert _relerr(g["u"], o["u"]) < 1e-12
    assert _relerr(g["w"], o["w"]) < 1e-12
    if mode != 0:
        assert (g["active"] == o["active"]).all()


@pytest.mark.parametrize("q", [2, 4, 8])
def test_parity_bounded_mask_and_order(gpu, q):
    sizes = [5, 40, 129, 12, 77, 600, 2, 33]
    rng = np.random.default_rng(7)
    bounded = (rng.random(sum(sizes)) < 0.7).astype(np.uint8)
    offs, g, o = _run(gpu, q, sizes, 2, seed=3, bounded=bounded, order="lpt")
    assert (g["status"] == 0).all()
    assert (g["active"] == o["active"]).all()
    assert not g["active"][bounded == 0].any()
    assert _relerr(g["u"], o["u"]) < 1e-12


@pytest.mark.parametrize("q", [2, 4, 8])
def test_mixed_precision_refinement(gpu, q):
    offs, g, o = _run(gpu, q, SIZES_RAGGED, 2, prec=1, seed=5)
    assert (g["status"] == 0).all(), g["status"]
    assert (g["active"] == o["active"]).all()
    assert _relerr(g["u"], o["u"]) < 1e-9


@pytest.mark.parametrize("q", [2, 4, 8])
def test_factor_then_solve(gpu, q):
    P = gpu
    sizes = [1, 2, 3, 6, 9, 50, 101, 256]
    offs, band, f = synth.lcp_batch(len(sizes), q, seed=11, sizes=sizes)
    rng = np.random.default_rng(1)
    pinned = (rng.random(len(f)) < 0.2).astype(np.uint8)
    dev = torch.device("cuda")
    bt = P.paqif.Batch(offs, q)
    pin_d = torch.as_tensor(pinned, device=dev)
    fac, st = P.paqif.factor(bt, torch.as_tensor(band, device=dev), pinned=pin_d)
    x = P.paqif.solve_factored(bt, fac, torch.as_tensor(f, device=dev), pinned=pin_d)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    x = x.cpu().numpy()
    for s in range(len(sizes)):
        a, b = offs[s], offs[s + 1]
        xo, sto = oracle.aqif_solve(band[a:b], f[a:b], pinned[a:b])
        assert sto == 0
        assert _relerr(x[a:b], xo) < 1e-12


@pytest.mark.parametrize("q", [2, 4, 8])
def test_factor_fp32_then_solve_and_refine(gpu, q):
    """FP32 factors (paqif_factor with PREC_FP32_IR): the FP32 solve against
    the oracle within 1e-4 relative, and FP64 iterative refinement with the
    FP32 solve as its correction step (residual b - A x formed in FP64 from
    the band) down to 1e-12.  Bound: FP32 unit roundoff 6e-8 times the
    growth of the elimination and the condition number of these strictly
    diagonally dominant systems (diagonal = sum |off-diagonal| + U(0.5, 1.5),
    so kappa_inf <= (2 (2q) + 1.5) / 0.5 < 70); each refinement step
    contracts the error by about kappa u_32 < 1e-5."""
    P = gpu
    sizes = [1, 2, 3, 6, 9, 50, 101, 256, 1025, 2049]
    offs, band, f = synth.lcp_batch(len(sizes), q, seed=12, sizes=sizes)
    rng = np.random.default_rng(2)
    pinned = (rng.random(len(f)) < 0.2).astype(np.uint8)
    dev = torch.device("cuda")
    bt = P.paqif.Batch(offs, q)
    pin_d = torch.as_tensor(pinned, device=dev)
    band_d = torch.as_tensor(band, device=dev)
    f_d = torch.as_tensor(f, device=dev)
    fac, st = P.paqif.factor(bt, band_d, pinned=pin_d, prec=P.PREC_FP32_IR)
    assert fac.numel() * fac.element_size() == bt.workspace_bytes(P.PREC_FP32_IR, P.LCP_LINEAR)
    x = P.paqif.solve_factored(bt, fac, f_d, pinned=pin_d, prec=P.PREC_FP32_IR)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    xo = np.zeros_like(f)
    for s in range(len(sizes)):
        a, b = offs[s], offs[s + 1]
        xo[a:b], sto = oracle.aqif_solve(band[a:b], f[a:b], pinned[a:b])
        assert sto == 0
    x0 = x.cpu().numpy()
    for s in range(len(sizes)):
        a, b = offs[s], offs[s + 1]
        e = _relerr(x0[a:b], xo[a:b])
        assert e < 1e-4, (s, e)
        assert e > 1e-12 or b - a < 50, (s, e)  # an FP32 solve, not the FP64 one
    # refinement: r = f_eff - A_eff x in FP64 (pinned rows: identity, rhs 0)
    bw = 2 * q + 1
    A_rows = band.reshape(-1, bw)
    x = x0.copy()
    for _ in range(4):
        r = np.zeros_like(f)
        for s in range(len(sizes)):
            a, b = int(offs[s]), int(offs[s + 1])
            n = b - a
            for i in range(n):
                gi = a + i
                if pinned[gi]:
                    r[gi] = -x[gi]
                    continue
                acc = f[gi]
                for d in range(bw):
                    j = i + d - q
                    if 0 <= j < n and not pinned[a + j]:
                        acc -= A_rows[gi, d] * x[a + j]
                r[gi] = acc
        dx = P.paqif.solve_factored(bt, fac, torch.as_tensor(r, device=dev), pinned=pin_d,
                                    prec=P.PREC_FP32_IR)
        x = x + dx.cpu().numpy()
    for s in range(len(sizes)):
        a, b = offs[s], offs[s + 1]
        assert _relerr(x[a:b], xo[a:b]) < 1e-12, s


def test_empty_and_zero_pivot(gpu):
    P = gpu
    dev = torch.device("cuda")
    # zero-size systems mixed with a singular one
    sizes = [0, 4, 0, 3]
    offs, band, f = synth.lcp_batch(len(sizes), 2, seed=2, sizes=sizes)
    band[4 + 1, :] = 0.0  # row 1 of the second non-empty system -> centre pivot 0
    bt = P.paqif.Batch(offs, 2)
    r = P.paqif.solve_lcp(bt, torch.as_tensor(band, device=dev), torch.as_tensor(f, device=dev),
                          mode=0)
    st = r["status"].cpu().numpy()
    assert st[0] == 0 and st[1] == 0 and st[2] == 0
    assert st[3] == 1  # SYS_ZERO_PIVOT


def test_invalid_arguments(gpu):
    P = gpu
    import ctypes
    bt = P.paqif.Batch([0, 5], 3)  # q = 3 unsupported
    n = P.lib().paqif_workspace_bytes(P.paqif.handle(), ctypes.byref(bt.c), 0, 2)
    assert n == 0
    band = torch.zeros(5 * 7, dtype=torch.float64, device="cuda")
    f = torch.zeros(5, dtype=torch.float64, device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    # the wrapper refuses it (its workspace query fails) ...
    with pytest.raises(ValueError):
        P.paqif.solve_lcp(bt, band, f, workspace=ws)
    # ... and so does the C ABI itself, before any launch
    u = torch.zeros(5, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    vp = ctypes.c_void_p
    code = P.lib().paqif_solve_lcp(P.paqif.handle(), ctypes.byref(bt.c), vp(band.data_ptr()),
                                   vp(f.data_ptr()), None, 2, 0, 1e-10, 64, vp(u.data_ptr()),
                                   None, None, vp(st.data_ptr()), None, vp(ws.data_ptr()), None)
    assert code == P._binding.PAQIF_EINVAL


def test_wrapper_refuses_short_buffers(gpu):
    """The C ABI takes bare pointers; the binding checks every per-row
    buffer and the workspace against the batch before calling it."""
    P = gpu
    offs, band, f = synth.lcp_batch(3, 2, seed=1, sizes=[10, 20, 30])
    bt = P.paqif.Batch(offs, 2)
    dev = torch.device("cuda")
    band_d = torch.as_tensor(band, device=dev)
    f_d = torch.as_tensor(f, device=dev)
    with pytest.raises(ValueError):
        P.paqif.solve_lcp(bt, band_d[:-1], f_d)
    with pytest.raises(ValueError):
        P.paqif.solve_lcp(bt, band_d, f_d[:-1])
    with pytest.raises(ValueError):
        P.paqif.solve_lcp(bt, band_d, f_d, bounded=torch.ones(59, dtype=torch.uint8, device=dev))
    # an FP32+IR workspace is smaller than an FP64 one: refused for FP64
    ws32 = bt.workspace(P.PREC_FP32_IR)
    assert ws32.numel() < bt.workspace_bytes(P.PREC_FP64)
    with pytest.raises(ValueError):
        P.paqif.solve_lcp(bt, band_d, f_d, prec=P.PREC_FP64, workspace=ws32)
    with pytest.raises(ValueError):
        P.paqif.factor(bt, band_d, factors=ws32)


def test_full_size_step_sampled(gpu):
    """The benchmark's step at full size: the three batches (q = 8, 4, 2,
    4096 systems each, n in [513, 4097]) in one paqif_solve_lcp_many call
    with the sweep counts its step tuning picks most often (16 / 16 / 12);
    the LCP certificate on every system, the largest and smallest systems
    and a random sample of each batch re-solved by the oracle."""
    P = gpu
    count = 4096
    dev = torch.device("cuda")
    data, calls = {}, []
    keep = {q: P.paqif.get_start_sweeps(q, 0) for q in (2, 4, 8)}
    try:
        for q, k in ((8, 12), (4, 16), (2, 16)):
            P.paqif.set_start_sweeps(q, 0, k)
            offs, band, f = synth.lcp_batch(count, q, seed=0)
            data[q] = (offs, band, f)
            bt = P.paqif.Batch(offs, q, order="lpt")
            calls.append(dict(batch=bt, band=torch.as_tensor(band, device=dev),
                              b=torch.as_tensor(f, device=dev)))
        print("full-size step, one solve_lcp_many call", flush=True)
        res = P.paqif.solve_lcp_many(calls, mode=P.LCP_EXACT)
        torch.cuda.synchronize()
    finally:
        for q, k in keep.items():
            P.paqif.set_start_sweeps(q, 0, k)
    for q, r in zip((8, 4, 2), res):
        offs, band, f = data[q]
        u = r["u"].cpu().numpy()
        w = r["w"].cpu().numpy()
        act = r["active"].cpu().numpy()
        assert (r["status"].cpu().numpy() == 0).all(), q
        scale = np.abs(f).max()
        assert u.min() >= 0.0
        assert (u[act == 1] == 0.0).all()
        assert w.min() >= -1e-12 * scale
        assert np.abs(u * w).max() <= 1e-12 * scale * max(1.0, np.abs(u).max())
        sizes = offs[1:] - offs[:-1]
        rng = np.random.default_rng(10 + q)
        pick = set(rng.choice(count, size=4, replace=False).tolist())
        pick |= {int(np.argmax(sizes)), int(np.argmin(sizes))}
        for s in sorted(pick):
            a, b = offs[s], offs[s + 1]
            o = oracle.lcp_solve(band[a:b], f[a:b])
            assert o["status"] == 0
            assert (o["active"] == act[a:b]).all(), (q, s)
            assert _relerr(u[a:b], o["u"]) < 1e-12, (q, s)


@pytest.mark.parametrize("q", [2, 4, 8])
def test_full_size_sampled(gpu, q):
    """Full-size workload (4096 systems, n in [513, 4097]) in the launch
    configuration the benchmark times; a sample of systems is re-solved by the
    oracle, and the LCP certificate is checked on every system."""
    P = gpu
    count = 4096
    offs, band, f = synth.lcp_batch(count, q, seed=0)
    dev = torch.device("cuda")
    bt = P.paqif.Batch(offs, q, order="lpt")
    band_d = torch.as_tensor(band, device=dev)
    f_d = torch.as_tensor(f, device=dev)
    r = P.paqif.solve_lcp(bt, band_d, f_d, mode=2)
    torch.cuda.synchronize()
    u = r["u"].cpu().numpy()
    w = r["w"].cpu().numpy()
    act = r["active"].cpu().numpy()
    st = r["status"].cpu().numpy()
    assert (st == 0).all()
    # certificate on all systems: u >= 0, w >= -tol, exact zeros on the active set
    scale = np.abs(f).max()
    assert u.min() >= 0.0
    assert (u[act == 1] == 0.0).all()
    assert w.min() >= -1e-12 * scale
    assert np.abs(u * w).max() <= 1e-12 * scale * max(1.0, np.abs(u).max())
    # sampled systems against the oracle
    rng = np.random.default_rng(q)
    for s in rng.choice(count, size=6, replace=False):
        a, b = offs[s], offs[s + 1]
        o = oracle.lcp_solve(band[a:b], f[a:b])
        assert o["status"] == 0
        assert (o["active"] == act[a:b]).all()
        assert _relerr(u[a:b], o["u"]) < 1e-12


@pytest.mark.parametrize("q", [2, 4, 8])
@pytest.mark.parametrize("prec", [0, 1])
def test_every_lane_layout(gpu, q, prec):
    """Each lane layout of the LCP kernel (selected by the autotuner at run
    time) gives the oracle's solution."""
    P = gpu
    sizes = [1, 2, 5, 8, 17, 64, 129, 300, 513, 1000]
    offs, band, f = synth.lcp_batch(len(sizes), q, seed=21, sizes=sizes)
    o = oracle.lcp_batch(q, offs, band, f, mode=2)
    bt = P.paqif.Batch(offs, q, order="lpt")
    dev = torch.device("cuda")
    band_d, f_d = torch.as_tensor(band, device=dev), torch.as_tensor(f, device=dev)
    keep = P.paqif.get_layout(q, prec)
    try:
        for lay in range(P.paqif.layout_count(q)):
            P.paqif.set_layout(q, prec, lay)
            r = P.paqif.solve_lcp(bt, band_d, f_d, mode=2, prec=prec)
            torch.cuda.synchronize()
            assert (r["status"].cpu().numpy() == 0).all(), lay
            assert (r["active"].cpu().numpy() == o["active"]).all(), lay
            tol = 1e-12 if prec == 0 else 1e-9
            assert _relerr(r["u"].cpu().numpy(), o["u"]) < tol, lay
    finally:
        P.paqif.set_layout(q, prec, keep)


def test_autotune_picks_a_layout(gpu):
    P = gpu
    offs, band, f = synth.lcp_batch(64, 4, seed=5)
    bt = P.paqif.Batch(offs, 4, order="lpt")
    dev = torch.device("cuda")
    chosen, times = P.paqif.autotune(bt, torch.as_tensor(band, device=dev),
                                     torch.as_tensor(f, device=dev))
    assert 0 <= chosen < P.paqif.layout_count(4)
    assert len(times) == P.paqif.layout_count(4) and min(times) > 0
    assert times[chosen] == min(times)


@pytest.mark.parametrize("q", [2, 4, 8])
@pytest.mark.parametrize("layout", [0, 1, 2, 3])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_layouts_modes_bounded_and_edges(gpu, q, layout, mode):
    """Every lane layout (q = 2 layout 2: one system per lane; layout 3: one
    system per 16-lane row group) in every mode, with a bounded mask, empty and
    one-row systems and a singular system."""
    P = gpu
    dev = torch.device("cuda")
    sizes = [0, 1, 7, 0, 64, 301, 3, 1000, 2, 17, 33]
    offs, band, f = synth.lcp_batch(len(sizes), q, seed=33 + q, sizes=sizes)
    rng = np.random.default_rng(5)
    bounded = (rng.random(len(f)) < 0.8).astype(np.uint8)
    sing = int(offs[6])  # the 3-row system: zero its centre row
    band[sing + 1, :] = 0.0
    o = oracle.lcp_batch(q, offs, band, f, mode=mode, bounded=bounded)
    bt = P.paqif.Batch(offs, q, order="lpt")
    keep = P.paqif.get_layout(q, 0)
    try:
        P.paqif.set_layout(q, 0, layout)
        r = P.paqif.solve_lcp(bt, torch.as_tensor(band, device=dev), torch.as_tensor(f, device=dev),
                              mode=mode, bounded=torch.as_tensor(bounded, device=dev))
        torch.cuda.synchronize()
    finally:
        P.paqif.set_layout(q, 0, keep)
    st = r["status"].cpu().numpy()
    assert (st == o["status"]).all(), (st, o["status"])
    u, act, w = r["u"].cpu().numpy(), r["active"].cpu().numpy(), r["w"].cpu().numpy()
    it = r["iters"].cpu().numpy()
    for s in range(len(sizes)):
        a, b = offs[s], offs[s + 1]
        if st[s] != 0 or b == a:
            continue
        assert (act[a:b] == o["active"][a:b]).all(), s
        assert 1 <= it[s] <= o["iters"][s] + 2, s
        assert _relerr(u[a:b], o["u"][a:b]) < 1e-12, s
        assert np.abs(w[a:b] - o["w"][a:b]).max() <= 1e-12 * max(1.0, np.abs(o["w"][a:b]).max())


@pytest.mark.parametrize("q", [2, 4, 8])
@pytest.mark.parametrize("layout", [0, 3])
@pytest.mark.parametrize("sweeps", [0, 1, 3, 8])
def test_start_sweeps_keep_the_solution(gpu, q, layout, sweeps):
    """The exact LCP's starting active set (projected Jacobi sweeps) changes
    the number of active-set solves, not the solution: active set and u
    against the oracle on ragged sizes with a bounded mask; with sweeps the
    largest systems need fewer solves than from the sign of b."""
    P = gpu
    dev = torch.device("cuda")
    sizes = [1, 2, 7, 64, 301, 1000, 2049, 2050, 1999]
    offs, band, f = synth.lcp_batch(len(sizes), q, seed=44 + q, sizes=sizes)
    rng = np.random.default_rng(q)
    bounded = (rng.random(len(f)) < 0.9).astype(np.uint8)
    o = oracle.lcp_batch(q, offs, band, f, mode=2, bounded=bounded)
    bt = P.paqif.Batch(offs, q, order="lpt")
    keep_l, keep_s = P.paqif.get_layout(q, 0), P.paqif.get_start_sweeps(q, 0)
    try:
        P.paqif.set_layout(q, 0, layout)
        P.paqif.set_start_sweeps(q, 0, sweeps)
        r = P.paqif.solve_lcp(bt, torch.as_tensor(band, device=dev), torch.as_tensor(f, device=dev),
                              mode=2, bounded=torch.as_tensor(bounded, device=dev))
        torch.cuda.synchronize()
    finally:
        P.paqif.set_layout(q, 0, keep_l)
        P.paqif.set_start_sweeps(q, 0, keep_s)
    assert (r["status"].cpu().numpy() == 0).all()
    assert (r["active"].cpu().numpy() == o["active"]).all()
    assert _relerr(r["u"].cpu().numpy(), o["u"]) < 1e-12
    it = r["iters"].cpu().numpy()
    if sweeps >= 8:
        big = np.array(sizes) >= 1999
        assert it[big].max() <= 2, it


@pytest.mark.parametrize("q", [2, 4, 8])
@pytest.mark.parametrize("sweeps", [1, 3, 8, 20])
def test_start_sweeps_iterate_matches_oracle(gpu, q, sweeps):
    """The start sweeps' kernel (workgroups of 512 held rows, several per
    system, one launch per 1 + 128/q sweeps) gives the oracle's starting
    active set: one active-set solve (max_iter = 1) from each side's A_0
    gives the same u (a start that differs in one row changes u there by the
    row's whole value).  Every system starts from the sweeps."""
    P = gpu
    dev = torch.device("cuda")
    sizes = [4097, 1, 2, 5, 700, 2049, 3001, 2868, 2866, 4000]
    offs, band, f = synth.lcp_batch(len(sizes), q, seed=70 + q, sizes=sizes)
    rng = np.random.default_rng(sweeps)
    bounded = (rng.random(len(f)) < 0.9).astype(np.uint8)
    start = oracle.lcp_start_sets(q, offs, band, f, bounded, k=sweeps, frac=0.0)
    bt = P.paqif.Batch(offs, q, order="lpt")
    keep = P.paqif.get_start_sweeps(q, 0)
    try:
        P.paqif.set_start_sweeps(q, 0, sweeps)
        print(f"start sweeps q={q} k={sweeps}", flush=True)
        r = P.paqif.solve_lcp(bt, torch.as_tensor(band, device=dev), torch.as_tensor(f, device=dev),
                              mode=2, max_iter=1, bounded=torch.as_tensor(bounded, device=dev))
        torch.cuda.synchronize()
    finally:
        P.paqif.set_start_sweeps(q, 0, keep)
    u = r["u"].cpu().numpy()
    st = r["status"].cpu().numpy()
    for s in range(len(sizes)):
        a, b = int(offs[s]), int(offs[s + 1])
        o = oracle.lcp_solve_start(band[a:b], f[a:b], bounded[a:b], start=start[a:b], max_iter=1)
        assert st[s] in (0, 3), (s, st[s])
        assert (st[s] == 0) == (o["status"] == 0), (s, st[s], o["status"])
        assert _relerr(u[a:b], o["u"]) < 1e-12, (s, sizes[s])


@pytest.mark.parametrize("q", [2, 4, 8])
@pytest.mark.parametrize("sweeps", [0, 3, 12, 20])
@pytest.mark.parametrize("prec", [0, 1])
def test_start_sweeps_split_matches_exact(gpu, q, sweeps, prec):
    """The start sweeps on their own (paqif_start_sweeps) followed by the
    solve from that iterate (LCP_EXACT_FROM_U) is one LCP_EXACT call split in
    two: the same u, w, active set, statuses and solve counts, bit for bit,
    with one sweep launch and two (q = 8 above 17 sweeps),
    and the sign start (0 sweeps: u = b); the oracle's active set too."""
    P = gpu
    dev = torch.device("cuda")
    sizes = [4097, 1, 2, 5, 700, 2049, 3001, 0, 2868, 513]
    offs, band, f = synth.lcp_batch(len(sizes), q, seed=90 + q, sizes=sizes)
    rng = np.random.default_rng(sweeps + 7)
    bounded = (rng.random(len(f)) < 0.9).astype(np.uint8)
    bt = P.paqif.Batch(offs, q, order="lpt")
    bd, fd = torch.as_tensor(band, device=dev), torch.as_tensor(f, device=dev)
    kd = torch.as_tensor(bounded, device=dev)
    keep = P.paqif.get_start_sweeps(q, prec)
    try:
        P.paqif.set_start_sweeps(q, prec, sweeps)
        print(f"split start q={q} k={sweeps} prec={prec}", flush=True)
        ref = P.paqif.solve_lcp(bt, bd, fd, mode=P.LCP_EXACT, prec=prec, bounded=kd)
        ws = bt.workspace(prec)
        u0 = P.paqif.start_sweeps(bt, bd, fd, prec=prec, bounded=kd, workspace=ws)
        got = P.paqif.solve_lcp(bt, bd, fd, mode=P.LCP_EXACT_FROM_U, prec=prec, bounded=kd,
                                workspace=ws, u=u0)
        torch.cuda.synchronize()
    finally:
        P.paqif.set_start_sweeps(q, prec, keep)
    assert got["u"].data_ptr() == u0.data_ptr()
    for k in ("u", "w", "active", "status", "iters"):
        assert torch.equal(got[k].cpu(), ref[k].cpu()), k
    st = got["status"].cpu().numpy()
    assert (st == 0).all(), st
    o = oracle.lcp_batch(q, offs, band, f, mode=oracle.EXACT, bounded=bounded)
    assert (got["active"].cpu().numpy() == o["active"]).all()


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_solve_lcp_many_matches_single_calls(gpu, mode, prec):
    """paqif_solve_lcp_many (every call's start sweeps, then the row-layout
    solves of all calls in one launch with their waves interleaved, the
    other layouts one kernel each) gives each call's paqif_solve_lcp result
    bit for bit: batches of q = 2, 4, 8 (ragged, up to 4097 rows, one with
    the same q twice, one empty), one of them on another lane layout."""
    P = gpu
    dev = torch.device("cuda")
    specs = [(8, [4097, 33, 1, 700, 2049, 5]), (2, [513, 4000, 2, 17, 0, 3001, 64]),
             (4, [2868, 9, 1500]), (2, [100, 257, 4097]), (4, []), (4, [65, 1025])]
    calls, singles = [], []
    keep_layout = P.paqif.get_layout(4, prec)
    try:
        for i, (q, sizes) in enumerate(specs):
            offs, band, f = synth.lcp_batch(len(sizes), q, seed=300 + i, sizes=sizes)
            rng = np.random.default_rng(i)
            bounded = (rng.random(len(f)) < 0.9).astype(np.uint8)
            bt = P.paqif.Batch(offs, q, order="lpt")
            bd, fd = torch.as_tensor(band, device=dev), torch.as_tensor(f, device=dev)
            kd = torch.as_tensor(bounded, device=dev)
            c = dict(batch=bt, band=bd, b=fd, bounded=kd)
            if mode == 3:
                c["u"] = P.paqif.start_sweeps(bt, bd, fd, prec=prec, bounded=kd)
            calls.append(c)
        # the last q = 4 call on the lane layout 0 (a kernel of its own)
        print(f"solve_lcp_many mode={mode} prec={prec}", flush=True)
        P.paqif.set_layout(4, prec, 3 if prec == 0 else 0)
        got = P.paqif.solve_lcp_many(calls[:5], mode=mode, prec=prec)
        P.paqif.set_layout(4, prec, 0)
        got += P.paqif.solve_lcp_many(calls[5:], mode=mode, prec=prec)
        P.paqif.set_layout(4, prec, 3 if prec == 0 else 0)
        for i, c in enumerate(calls):
            if i == 5:
                P.paqif.set_layout(4, prec, 0)
            if mode == 3:  # the many-call solve overwrote u: start again
                c["u"] = P.paqif.start_sweeps(c["batch"], c["band"], c["b"], prec=prec,
                                              bounded=c["bounded"])
            singles.append(P.paqif.solve_lcp(c["batch"], c["band"], c["b"], mode=mode, prec=prec,
                                             bounded=c["bounded"], u=c.get("u")))
        torch.cuda.synchronize()
    finally:
        P.paqif.set_layout(4, prec, keep_layout)
    for i, (g, r) in enumerate(zip(got, singles)):
        for k in ("u", "w", "active", "status", "iters"):
            assert torch.equal(g[k].cpu(), r[k].cpu()), (i, k)
        assert (g["status"].cpu().numpy() == 0).all(), (i, g["status"])
    assert P.paqif.solve_lcp_many([], mode=mode, prec=prec) == []


def test_solve_lcp_many_argument_checks(gpu):
    P = gpu
    dev = torch.device("cuda")
    offs, band, f = synth.lcp_batch(2, 2, seed=5, sizes=[10, 20])
    bt = P.paqif.Batch(offs, 2)
    c = dict(batch=bt, band=torch.as_tensor(band, device=dev), b=torch.as_tensor(f, device=dev))
    with pytest.raises(ValueError):
        P.paqif.solve_lcp_many([c] * 9)
    with pytest.raises(ValueError):
        P.paqif.solve_lcp_many([c], mode=P.LCP_EXACT_FROM_U)
    with pytest.raises(RuntimeError):
        P.paqif.solve_lcp_many([c], mode=7)
    with pytest.raises(RuntimeError):
        P.paqif.solve_lcp_many([c], max_iter=0)


def test_start_from_u_argument_checks(gpu):
    P = gpu
    dev = torch.device("cuda")
    offs, band, f = synth.lcp_batch(3, 2, seed=5, sizes=[10, 20, 7])
    bt = P.paqif.Batch(offs, 2)
    bd, fd = torch.as_tensor(band, device=dev), torch.as_tensor(f, device=dev)
    with pytest.raises(ValueError):
        P.paqif.solve_lcp(bt, bd, fd, mode=P.LCP_EXACT_FROM_U)
    with pytest.raises(ValueError):
        P.paqif.solve_lcp(bt, bd, fd, mode=P.LCP_EXACT, u=torch.zeros_like(fd))
    with pytest.raises(ValueError):
        P.paqif.start_sweeps(bt, bd, fd, u=torch.zeros(5, dtype=torch.float64, device=dev))
    with pytest.raises(RuntimeError):  # max_iter < 1 is rejected by the library
        P.paqif.solve_lcp(bt, bd, fd, mode=P.LCP_EXACT_FROM_U, u=torch.zeros_like(fd),
                          max_iter=0)


def test_start_sweeps_argument_checks(gpu):
    P = gpu
    with pytest.raises(RuntimeError):
        P.paqif.set_start_sweeps(4, 0, 33)
    with pytest.raises(RuntimeError):
        P.paqif.set_start_sweeps(3, 0, 2)
    keep = P.paqif.get_start_sweeps(4, 1)
    P.paqif.set_start_sweeps(4, 1, 6)
    assert P.paqif.get_start_sweeps(4, 1) == 6
    P.paqif.set_start_sweeps(4, 1, keep)


@pytest.mark.parametrize("q", [2, 8])
def test_start_sweeps_fp32_refined(gpu, q):
    offs, g, o = _run(gpu, q, SIZES_RAGGED + [2049], 2, prec=1, seed=9)
    assert (g["status"] == 0).all(), g["status"]
    assert (g["active"] == o["active"]).all()
    assert _relerr(g["u"], o["u"]) < 1e-9
