"""Benchmark: batched PAQIF banded-LCP solves/s on one MI355X.

Workload (synthetic, seeded; stands in for the paper's unpublished matrices):
three batches of 4096 symmetric, strictly diagonally dominant band systems,
orders uniform in [513, 4097], half-bandwidth q = 2, 4 and 8, off-diagonals
U(-1, 1), diagonal = sum|off-diagonals| + U(0.5, 1.5), right-hand side
N(0, 1).  One step = the exact LCP solve (active-set PAQIF, FP64) of all three
batches, 12288 solves; inputs are resident in HBM before timing starts.

Prints one JSON line.  ``--gpus`` above 1 is refused: the benchmark runs on
one GPU (batches would shard by total rows across GPUs with no exchange).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNT = 4096
QS = (2, 4, 8)


def algorithmic_bytes_per_row(q):
    # band 8(2q+1) + b 8 + u 8 + Z0 written and read back 2*8(2q+1), per
    # active-set iteration (the per-row unit of the LCP solve)
    return 8 * (2 * q + 1) + 8 + 8 + 2 * 8 * (2 * q + 1)


def mixed_bytes_per_row(q):
    # FP32 + refinement, per active-set iteration: FP64 band 8(2q+1), b and u,
    # FP32 level records Z (4q+6 values per level, ~ (2q+3) per row) and W
    # multipliers (4q per level, 2q per row) written and read back once;
    # the refinement sweeps' extra residual and re-solve traffic is not
    # counted (the kernel does not report their number)
    return 8 * (2 * q + 1) + 8 + 8 + 2 * 4 * ((2 * q + 3) + 2 * q)


def lcp_call_kernels(P, q, prec):
    """Kernels of one exact paqif_solve_lcp call: the start sweeps (if the
    handle runs any) and the solve."""
    k = lcp_kernel_name(P, q, prec)
    if P.paqif.get_start_sweeps(q, prec) > 0:
        k = f"paqif_sweep_kernel<{q}> + " + k
    return k


def lcp_kernel_name(P, q, prec):
    """Name of the solve kernel paqif_solve_lcp launches for (q, prec) under
    the handle's current lane layout."""
    lay = P.paqif.get_layout(q, prec)
    if prec == P.PREC_FP64 and lay == 3:
        return f"paqif_lcp_rows_kernel<{q}>"
    if prec == P.PREC_FP64 and lay == 2 and q == 2:
        return "paqif_lcp_lane_kernel<2>"
    if prec != P.PREC_FP64 and (lay == 3 or (lay == 2 and q == 2)):
        lay = 0
    return f"paqif_lcp_kernel<{q},{lay},{'double' if prec == P.PREC_FP64 else 'float'}>"


def sweep_bytes(q, sizes, sweeps):
    """Algorithmic bytes of the exact LCP's start sweeps (projected Jacobi
    from u = 0, paqif_sweep_kernel): its launches run up to 1 + 128/q sweeps
    each with the band rows held on chip, so per row and launch the band
    8(2q+1), b and the iterate written, plus the previous iterate read by
    every launch after the first; every system is swept."""
    if sweeps <= 0:
        return 0
    launches = -(-sweeps // (1 + 128 // q))
    rows = int(sizes.sum())
    return rows * (launches * (8 * (2 * q + 1) + 16) + (launches - 1) * 8)


def minimum_bytes_per_row(q):
    # band, b and u read once per active-set iteration (no factor traffic)
    return 8 * (2 * q + 1) + 8 + 8


def copy_bandwidth(torch):
    # device copy of 2^25 doubles (read + write), HIP events, best of 5
    src = torch.rand(1 << 25, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2 * (1 << 25) * 8 / (best / 1e3) / 1e9


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def deformation_leg(P, torch, args):
    """MFMA use of the elastic deformation (2N^2 B flops for a line grid,
    2 (Nx Ny)^2 B for a point grid): N = 4097 with B = 170 instances (the
    largest sweep group) and the 257 x 257 point grid, B = 1, in each
    precision the library offers; HIP events, median of 5."""
    # precision codes of the library: 0 FP64, 3 FP32, 2 split BF16 (three
    # BF16 products per FP32-like product; flops counted algorithmically)
    peaks = {0: 78.6, 3: 157.3, 2: 2500.0}
    names = {0: "fp64", 3: "fp32", 2: "split_bf16"}
    out = {}
    for tag, grid, shape, flops in (
            ("line_N4097_B170", P.ehl.line_grid(4097), (170, 4097), 2.0 * 4097 ** 2 * 170),
            ("point_257x257", P.ehl.point_grid(257, 257), (1, 257, 257), 2.0 * (257 * 257) ** 2)):
        Pf = torch.rand(shape, dtype=torch.float64, device="cuda")
        res = {}
        for prec in (0, 3, 2):
            try:
                P.ehl.deformation(Pf, grid, prec=prec)
            except (RuntimeError, ValueError):
                continue
            ts = []
            for _ in range(5):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                P.ehl.deformation(Pf, grid, prec=prec)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            tf = flops / (ms / 1e3) / 1e12
            res[names[prec]] = dict(ms=round(ms, 4), tflops=round(tf, 2),
                                    peak_tflops=peaks[prec], frac=round(tf / peaks[prec], 4))
        out[tag] = res
        log(f"deformation {tag}: " + ", ".join(f"{k} {v['ms']} ms ({v['frac']:.1%})"
                                               for k, v in res.items()))
    return out


def active30_leg(P, torch, synth, args):
    """Config 2 with b ~ N(0.55, 1) (about 30 % active): one warm-up and
    three timed solves per q, FP64 exact LCP."""
    out = {}
    tot_ms = 0.0
    for q in QS:
        offs, band, f = synth.lcp_batch(COUNT, q, seed=args.seed, rhs_mean=0.55)
        bt = P.paqif.Batch(offs, q, order="lpt")
        bd = torch.as_tensor(band, device="cuda")
        fd = torch.as_tensor(f, device="cuda")
        ws = bt.workspace(P.PREC_FP64)
        r = P.paqif.solve_lcp(bt, bd, fd, mode=P.LCP_EXACT, workspace=ws)
        ts = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            r = P.paqif.solve_lcp(bt, bd, fd, mode=P.LCP_EXACT, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.mean(ts))
        tot_ms += ms
        out[str(q)] = dict(avg_ms=round(ms, 4), active_frac=round(float(r["active"].float().mean()), 4),
                           iters_mean=round(float(r["iters"].float().mean()), 3),
                           status_ok=bool((r["status"] == 0).all().item()))
        del bd, fd, ws
    out["solves_per_s"] = round(len(QS) * COUNT / (tot_ms / 1e3), 1)
    log(f"config 2 at ~30% active: {out['solves_per_s']:.0f} solves/s")
    return out


def cpu_baseline(batches, sample, nthreads):
    import oracle
    t_total = 0.0
    solves = 0
    for q, (offs, band, f) in batches.items():
        so = offs[: sample + 1]
        nrow = int(so[-1])
        t0 = time.perf_counter()
        oracle.lcp_batch(q, so, band[:nrow], f[:nrow], mode=oracle.EXACT, nthreads=nthreads)
        t_total += time.perf_counter() - t0
        solves += sample
    return solves / t_total


def measured_traffic(kernel_q, kernel):
    """HBM bytes of one exact solve call at this q (summed over its kernels)
    from the committed counter summary, if it was taken on these kernels and
    the current kernel sources (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "paqif_lcp_q8_hbm_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_val = re.search(rf"traffic_bytes_per_call_q{kernel_q}_fp64:\s*([0-9.eE+]+)", txt)
    m_ker = re.search(rf"traffic_kernels_q{kernel_q}:\s*(\S+)", txt)
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", txt)
    if not (m_val and m_sha and m_ker) or m_ker.group(1) != kernel:
        return None
    h = hashlib.sha256()
    for f in ("paqif.hip", "common.h", "paqif_args.h"):
        h.update(open(os.path.join(ROOT, "paper_2008_03276_amd", "csrc", f), "rb").read())
    return float(m_val.group(1)) if h.hexdigest() == m_sha.group(1) else None


def measured_step_traffic(kernels):
    """HBM bytes of one step of the default (one-call) mode, summed over its
    kernels, from the committed counter summary, if it was taken on these
    kernels and the current kernel sources (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "paqif_lcp_q8_hbm_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_val = re.search(r"traffic_bytes_per_step_fp64:\s*([0-9.eE+]+)", txt)
    m_ker = re.search(r"traffic_kernels_step:\s*(\S+)", txt)
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", txt)
    if not (m_val and m_sha and m_ker) or m_ker.group(1) != kernels:
        return None
    h = hashlib.sha256()
    for f in ("paqif.hip", "common.h", "paqif_args.h"):
        h.update(open(os.path.join(ROOT, "paper_2008_03276_amd", "csrc", f), "rb").read())
    return float(m_val.group(1)) if h.hexdigest() == m_sha.group(1) else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def ehl_legs(P, torch, synth, dev, args):
    """EHL solves/s: config 1 (N=257, M=20, L=10, one instance, time to
    solution) and a batched line-contact sweep (M log-uniform in [10,1000],
    L uniform in [5,20], N in {1025, 2049, 4097}, one batch per N) in FP64,
    plus the FP32-deformation (+FP64 refresh) variant on the N=1025 batch;
    iterations and statuses reported."""
    import time as _t
    out = {}
    # config 1
    P.ehl.solve_line([20.0], [10.0], 257)  # warm-up (graph instantiation etc.)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    r = P.ehl.solve_line([20.0], [10.0], 257)
    torch.cuda.synchronize()
    dt = _t.perf_counter() - t0
    log(f"ehl config1 done in {dt:.3f} s")
    out["config1"] = dict(seconds=round(dt, 4), solves_per_s=round(1.0 / dt, 3),
                          status=int(r["status"][0]), newton_steps=int(r["iters"][0]),
                          H0=float(r["H0"][0]), Hmin=float(r["Hmin"][0]))
    if not args.no_cpu:
        # the oracle (numpy, one process) on the same instance
        from oracle import ehl_line as OE
        t0 = _t.perf_counter()
        ro = OE.solve_line(20.0, 10.0, 257)
        out["config1"]["oracle"] = dict(seconds=round(_t.perf_counter() - t0, 3),
                                        status=int(ro["status"]), newton_steps=int(ro["iters"]))
    # the same contact with the kappa-scheme convection instead of van Leer
    kap = {}
    for kappa in (0.0, 1.0 / 3.0, -1.0):
        o = P.ehl.default_opts(convection=1, kappa=kappa)
        P.ehl.solve_line([20.0], [10.0], 257, opts=o)
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        r = P.ehl.solve_line([20.0], [10.0], 257, opts=o)
        torch.cuda.synchronize()
        kap[f"kappa_{kappa:.3f}"] = dict(seconds=round(_t.perf_counter() - t0, 4),
                                         status=int(r["status"][0]),
                                         newton_steps=int(r["iters"][0]),
                                         H0=float(r["H0"][0]), Hmin=float(r["Hmin"][0]))
    out["config1_kappa_scheme"] = kap
    # sweep: nb instances, N drawn from {1025, 2049, 4097} (grouped by N,
    # one batched solve per group), FP64; the FP32-deformation variant
    # (+ FP64 refresh) on the N = 1025 group
    nb = args.ehl_sweep
    M, L = synth.ehl_sweep_params(nb, seed=args.seed)
    groups = np.array_split(np.arange(nb), 3)
    res = {"instances": nb, "groups": {}}
    t_all, conv_all = 0.0, 0
    P1025 = None
    for N, idx in zip((1025, 2049, 4097), groups):
        # active-set cap 8: a warm-started step's LCP needs about one solve,
        # and a batched launch lasts as long as its slowest (cycling) system;
        # an instance whose change sets no new minimum in 600 steps stops
        opts = P.ehl.default_opts(max_newton=3000, lcp_max_iter=8, stall_steps=600)
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        r = P.ehl.solve_line(M[idx], L[idx], N, opts=opts)
        torch.cuda.synchronize()
        dt = _t.perf_counter() - t0
        st = r["status"].cpu().numpy()
        it = r["iters"].cpu().numpy()
        ok = st == 0
        res["groups"][str(N)] = dict(
            instances=int(len(idx)), seconds=round(dt, 3), converged=int(ok.sum()),
            statuses={str(int(k)): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
            mean_newton_steps_converged=float(it[ok].mean()) if ok.any() else None)
        t_all += dt
        conv_all += int(ok.sum())
        if N == 1025:
            P1025, ok1025, idx1025 = r["P"], ok, idx
        if N == 4097:
            st4097, idx4097 = st, idx
        log(f"ehl sweep N={N}: {dt:.2f} s, converged {int(ok.sum())}/{len(idx)}")
    res.update(seconds=round(t_all, 3), converged=conv_all, failed=nb - conv_all,
               converged_per_s=round(conv_all / t_all, 3),
               all_instances_per_s=round(nb / t_all, 3))
    # the N = 4097 instances that stopped on the active-set cap of 8, re-run
    # once with the library default cap of 64: do they converge, or cycle?
    capped = idx4097[st4097 == 3] if args.sweep_cap64 else idx4097[:0]
    if len(capped):
        opts64 = P.ehl.default_opts(max_newton=3000, lcp_max_iter=64, stall_steps=600)
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        r = P.ehl.solve_line(M[capped], L[capped], 4097, opts=opts64)
        torch.cuda.synchronize()
        st64 = r["status"].cpu().numpy()
        res["N4097_cap8_failures_at_cap64"] = dict(
            instances=int(len(capped)), seconds=round(_t.perf_counter() - t0, 3),
            statuses={str(int(k)): int(v) for k, v in zip(*np.unique(st64, return_counts=True))})
        log(f"ehl sweep N=4097 cap-8 failures at cap 64: {res['N4097_cap8_failures_at_cap64']}")
    if not args.no_cpu:
        # the oracle on a seeded subset: the first instance of the N = 1025
        # group (the full sweep would take the oracle hours)
        from oracle import ehl_line as OE
        i0 = int(idx1025[0])
        t0 = _t.perf_counter()
        ro = OE.solve_line(float(M[i0]), float(L[i0]), 1025, max_newton=3000, stall_steps=600)
        res["oracle_subset"] = dict(instances=1, N=1025, M=float(M[i0]), L=float(L[i0]),
                                    seconds=round(_t.perf_counter() - t0, 3),
                                    status=int(ro["status"]), newton_steps=int(ro["iters"]),
                                    gpu_seconds_per_instance_in_batch=round(
                                        res["groups"]["1025"]["seconds"] / len(idx1025), 4))
    opts = P.ehl.default_opts(deform_prec=P.PREC_FP32, max_newton=3000, lcp_max_iter=8,
                              stall_steps=600)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    r = P.ehl.solve_line(M[idx1025], L[idx1025], 1025, opts=opts)
    torch.cuda.synchronize()
    dt = _t.perf_counter() - t0
    ok32 = r["status"].cpu().numpy() == 0
    both = torch.as_tensor(ok32 & ok1025, device=r["P"].device)
    d = None
    if bool(both.any()):
        p64, p32 = P1025[both], r["P"][both]
        d = float(((p32 - p64).abs().amax(dim=1) / p64.abs().amax(dim=1)).max())
    res["fp32_deform_N1025"] = dict(seconds=round(dt, 3), converged=int(ok32.sum()),
                                    fp64_seconds=res["groups"]["1025"]["seconds"],
                                    max_rel_diff_vs_fp64=d, compared_instances=int(both.sum()))
    log(f"ehl sweep N=1025 FP32 deformation: {dt:.2f} s, converged {int(ok32.sum())}")
    out["sweep"] = res
    if not args.no_adjoint:
        out["adjoint_N2049"] = adjoint_leg(P, torch, synth, args)
    if not args.no_point:
        out[f"point_{args.point_n}"] = point_leg(P, torch, args)
    out["convdiff"] = convdiff_leg(P, torch, args)
    return out


def convdiff_leg(P, torch, args):
    """Convection-diffusion workload (linear case study of the numerical
    results): 257 x 257 nodes, eps = 1e-6, kappa in {0, 1/3, -1}, line
    relaxation to max defect <= 1e-10 max|f|; iterations, time, line solves
    per second and the max error against x^4 + y^4.  With the CPU leg on, the
    oracle's time at 65 x 65 nodes beside the GPU's at the same size."""
    import time as _t
    out = {}
    x = None
    for n in (257, 65):
        x = np.linspace(-1.0, 1.0, n)
        ex = x[:, None] ** 4 + x[None, :] ** 4
        ws = torch.empty(P.lib().cd_workspace_bytes(n), dtype=torch.uint8, device="cuda")
        res_n = {}
        for kappa in (0.0, 1.0 / 3.0, -1.0):
            f, u = P.convdiff.example(n)
            P.convdiff.line_relax(f, u.clone(), kappa, tol=1e-10, max_iter=2, workspace=ws)
            torch.cuda.synchronize()
            t0 = _t.perf_counter()
            it, res = P.convdiff.line_relax(f, u, kappa, tol=1e-10, max_iter=2000, workspace=ws)
            torch.cuda.synchronize()
            dt = _t.perf_counter() - t0
            err = float(np.abs(u.cpu().numpy() - ex)[1:-1, 1:-1].max() / ex[1:-1, 1:-1].max())
            res_n[f"kappa_{kappa:.3f}"] = dict(
                iterations=it, ms=round(dt * 1e3, 3), ms_per_iteration=round(dt * 1e3 / it, 4),
                line_solves_per_s=round(2 * (n - 2) * it / dt, 1), max_defect=res,
                linf_rel_error=err)
        out[f"n{n}"] = res_n
        log(f"convdiff n={n}: " + ", ".join(f"{k} {v['iterations']} it {v['ms']} ms"
                                             for k, v in res_n.items()))
    # the distributive line relaxation (Ls3) on 65 x 65 nodes: the paper's
    # warning that it is not robust shows as slow convergence
    n = 65
    ws3 = torch.empty(P.lib().cd_ls3_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    ls3 = {}
    for kappa in (0.0, 1.0 / 3.0, -1.0):
        f, u = P.convdiff.example(n)
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        it, res = P.convdiff.distributive_relax(f, u, kappa, tol=1e-10, max_iter=2000,
                                                workspace=ws3)
        torch.cuda.synchronize()
        dt = _t.perf_counter() - t0
        fmax = float(f[1:-1, 1:-1].abs().max())
        ls3[f"kappa_{kappa:.3f}"] = dict(iterations=it, ms=round(dt * 1e3, 3),
                                         ms_per_iteration=round(dt * 1e3 / it, 4),
                                         rel_defect=res / fmax, converged=bool(res <= 1e-10 * fmax))
    out["ls3_n65"] = ls3
    log("convdiff Ls3 n=65: " + ", ".join(f"{k} {v['iterations']} it rel. defect {v['rel_defect']:.1e}"
                                          for k, v in ls3.items()))
    # the paper's x-line splittings Ls0 / Ls1 (two colours per sweep, omega
    # 0.7) on 65 x 65 and 257 x 257 nodes, at most 2000 sweeps
    for n in (65, 257):
        ws = torch.empty(P.lib().cd_workspace_bytes(n), dtype=torch.uint8, device="cuda")
        spl = {}
        for which in (0, 1):
            for kappa in (0.0, 1.0 / 3.0, -1.0):
                f, u = P.convdiff.example(n)
                torch.cuda.synchronize()
                t0 = _t.perf_counter()
                it, res = P.convdiff.split_relax(f, u, which, kappa, omega=0.7, tol=1e-10,
                                                 max_iter=2000, workspace=ws)
                torch.cuda.synchronize()
                dt = _t.perf_counter() - t0
                fmax = float(f[1:-1, 1:-1].abs().max())
                spl[f"Ls{which}_kappa_{kappa:.3f}"] = dict(
                    iterations=it, ms=round(dt * 1e3, 3), ms_per_iteration=round(dt * 1e3 / it, 4),
                    rel_defect=res / fmax, converged=bool(res <= 1e-10 * fmax))
        out[f"ls01_n{n}"] = spl
        log(f"convdiff Ls0/Ls1 n={n}: " + ", ".join(
            f"{k} {v['iterations']} it {v['rel_defect']:.1e}" for k, v in spl.items()))
    if not args.no_cpu:
        from oracle import convdiff as OC
        cpu = {}
        for kappa in (0.0, 1.0 / 3.0, -1.0):
            t0 = _t.perf_counter()
            r = OC.solve(65, kappa, tol=1e-10, max_iter=2000)
            cpu[f"kappa_{kappa:.3f}"] = dict(iterations=r["iters"],
                                             ms=round((_t.perf_counter() - t0) * 1e3, 1))
        out["oracle_n65"] = cpu
    return out


def partitioned_leg(P, torch, synth, args):
    """Partitioned PAQIF of one long band system (n = 2^20 and 2^22 rows,
    q = 2 and 4, linear mode): time per solve over r blocks (HIP events on
    the library's stream, median of 5 after one warm-up), against the same
    kernel on the unpartitioned system (one wavefront walks n/2 levels) and,
    with the CPU leg on, the oracle's serial AQIF solve of the same system."""
    import time as _t
    out = {}
    cases = ((1 << 20, 2, (256, 512, 1024, 2048, 4096)),
             (1 << 20, 4, (128, 256, 512, 1024)),
             (1 << 22, 2, (512, 1024, 2048, 4096, 8192)))
    if args.part_case:  # one (n, q, r) only, no unpartitioned or CPU run (for profiling)
        n_, q_, r_ = (int(v) for v in args.part_case.split(":"))
        cases = ((n_, q_, (r_,)),)
    for n, q, rs in cases:
        band_h, f_h = synth.long_system(n, q, seed=args.seed)
        band = torch.as_tensor(band_h, device="cuda")
        f = torch.as_tensor(f_h, device="cuda")
        res = {}
        for r in rs:
            ws = torch.empty(P.paqif.partitioned_workspace_bytes(n, q, r), dtype=torch.uint8,
                             device="cuda")
            res_p = P.paqif.solve_partitioned(band, f, r, workspace=ws)
            times = []
            for _ in range(5):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                res_p = P.paqif.solve_partitioned(band, f, r, workspace=ws)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            res[str(r)] = dict(ms=round(float(np.median(times)), 4),
                               status=int(res_p["status"].cpu()[0]))
            del ws
        best = min(res, key=lambda k: res[k]["ms"])
        entry = dict(n=n, q=q, r=res, best_r=int(best), best_ms=res[best]["ms"],
                     rows_per_s=round(n / (res[best]["ms"] / 1e3), 1),
                     layout=P.paqif.get_layout(q))
        if not args.part_case:
            # the block solves at the best r with each lane layout of the kernel
            keep = P.paqif.get_layout(q)
            ws = torch.empty(P.paqif.partitioned_workspace_bytes(n, q, int(best)),
                             dtype=torch.uint8, device="cuda")
            lay = {}
            for L in range(P.paqif.layout_count(q)):
                P.paqif.set_layout(q, P.PREC_FP64, L)
                P.paqif.solve_partitioned(band, f, int(best), workspace=ws)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                P.paqif.solve_partitioned(band, f, int(best), workspace=ws)
                e1.record()
                torch.cuda.synchronize()
                lay[str(L)] = round(e0.elapsed_time(e1), 4)
            P.paqif.set_layout(q, P.PREC_FP64, keep)
            entry["ms_by_layout_at_best_r"] = lay
            # the same solve replayed from a captured graph (launch overhead
            # of its ~10 kernels removed)
            st_ = torch.cuda.Stream()
            st_.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st_):
                P.paqif.solve_partitioned(band, f, int(best), workspace=ws)
            torch.cuda.current_stream().wait_stream(st_)
            torch.cuda.synchronize()
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr):
                P.paqif.solve_partitioned(band, f, int(best), workspace=ws)
            gr.replay()
            gts = []
            for _ in range(5):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                gr.replay()
                e1.record()
                torch.cuda.synchronize()
                gts.append(e0.elapsed_time(e1))
            entry["graph_replay_ms_at_best_r"] = round(float(np.median(gts)), 4)
            del gr
            del ws
        if n == 1 << 20 and not args.part_case:
            # the unpartitioned system alone: lane layout 0 (a wavefront per system)
            keep = P.paqif.get_layout(q)
            P.paqif.set_layout(q, P.PREC_FP64, 0)
            bt = P.paqif.Batch(np.array([0, n], dtype=np.int64), q)
            ws1 = bt.workspace(P.PREC_FP64, P.LCP_LINEAR)
            P.paqif.solve_lcp(bt, band, f, mode=P.LCP_LINEAR, workspace=ws1, want_w=False,
                              want_active=False)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            r1 = P.paqif.solve_lcp(bt, band, f, mode=P.LCP_LINEAR, workspace=ws1, want_w=False,
                                   want_active=False)
            e1.record()
            torch.cuda.synchronize()
            mono = e0.elapsed_time(e1)
            P.paqif.set_layout(q, P.PREC_FP64, keep)
            u = P.paqif.solve_partitioned(band, f, int(best))["u"]
            # the exact LCP (eq. 14) by the active-set iteration around the
            # partitioned solve (host-synchronised after each solve)
            P.paqif.solve_partitioned(band, f, int(best), mode=P.LCP_EXACT)
            t0 = _t.perf_counter()
            rx = P.paqif.solve_partitioned(band, f, int(best), mode=P.LCP_EXACT)
            torch.cuda.synchronize()
            entry["exact"] = dict(ms=round((_t.perf_counter() - t0) * 1e3, 3),
                                  solves=int(rx["iters"].cpu()[0]),
                                  status=int(rx["status"].cpu()[0]),
                                  active_frac=round(float(rx["active"].float().mean()), 4))
            d = float((u - r1["u"]).abs().max() / r1["u"].abs().max())
            entry["unpartitioned_ms"] = round(mono, 3)
            entry["speedup_vs_unpartitioned"] = round(mono / res[best]["ms"], 1)
            entry["max_rel_diff_vs_unpartitioned"] = d
            del ws1
            if not args.no_cpu:
                import oracle
                t0 = _t.perf_counter()
                oracle.aqif_solve(band_h, f_h)
                entry["oracle_serial_ms"] = round((_t.perf_counter() - t0) * 1e3, 2)
                t0 = _t.perf_counter()
                ro = oracle.lcp_solve(band_h, f_h, mode=oracle.EXACT, max_iter=64)
                entry["exact"]["oracle_serial_ms"] = round((_t.perf_counter() - t0) * 1e3, 2)
                entry["exact"]["oracle_solves"] = int(ro["iters"])
        out[f"n{n}_q{q}"] = entry
        log(f"partitioned n={n} q={q}: best r={best} {res[best]['ms']:.3f} ms"
            + (f", unpartitioned {entry['unpartitioned_ms']:.1f} ms"
               if "unpartitioned_ms" in entry else ""))
        del band, f
        torch.cuda.empty_cache()
    return out


def adjoint_leg(P, torch, synth, args):
    """Adjoint of the line contact: N=2049, 64 instances, M log-uniform in
    [20, 500], L = 10, roughness A sin(2 pi X / 0.25).  Forward solve, then
    the hand-written adjoint for out = H0 (gH0 = 1) and out = Hmin (film
    cotangent at the arg-min); gradients dM, dL and d(roughness)."""
    import time as _t
    NN, B = 2049, 64
    M, L = synth.ehl_adjoint_params(B, seed=args.seed)
    x = -4.5 + 6.0 * np.arange(NN) / (NN - 1)
    dev = torch.device("cuda", 0)
    rg = torch.as_tensor(np.stack([synth.roughness(x, amplitude=args.rough_amp)] * B), device=dev)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    r = P.ehl.solve_line(M, L, NN, rough=rg)
    torch.cuda.synchronize()
    t_fwd = _t.perf_counter() - t0
    ok = (r["status"] == 0)
    gH = torch.zeros_like(r["H"])
    gH[torch.arange(B, device=dev), torch.argmin(r["H"], dim=1)] = 1.0
    ones = torch.ones(B, dtype=torch.float64, device=dev)
    P.ehl.adjoint(M, L, NN, r["P"], r["H0"], gH0=ones, rough=rg)  # warm-up
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    a0 = P.ehl.adjoint(M, L, NN, r["P"], r["H0"], gH0=ones, rough=rg)
    a1 = P.ehl.adjoint(M, L, NN, r["P"], r["H0"], gH=gH, rough=rg)
    torch.cuda.synchronize()
    t_adj = _t.perf_counter() - t0
    okn = ok.cpu().numpy()
    st0, st1 = a0["status"].cpu().numpy(), a1["status"].cpu().numpy()
    log(f"adjoint leg: forward {t_fwd:.2f} s ({int(okn.sum())}/{B} converged), "
        f"adjoint {t_adj:.3f} s")
    return dict(forward_seconds=round(t_fwd, 3), converged=int(okn.sum()), instances=B,
                roughness_amplitude=args.rough_amp,
                adjoint_seconds_two_outputs=round(t_adj, 4),
                gradients_per_s=round(2 * B / t_adj, 2),
                adjoint_status_ok_on_converged=bool((st0[okn] == 0).all() and (st1[okn] == 0).all()),
                arnoldi_steps_mean=float((a0["iters"].float().mean() + a1["iters"].float().mean()) / 2),
                example=dict(M=float(M[0]), dH0_dM=float(a0["dM"][0]), dHmin_dL=float(a1["dL"][0])))


def point_leg(P, torch, args):
    """Point contact: n x n nodes (257 by default) on [-4.5, 1.5] x [-3, 3], M = 200,
    L = 10, load 2 pi/3; alternating two-colour x/y line sweeps to
    max |dP| <= 1e-10 per step; time to solution."""
    import time as _t
    opts = P.ehl.default_opts(tol=1e-10, max_newton=30000, c_h0=0.02)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    n = args.point_n
    r = P.ehl.solve_point([200.0], [10.0], n, n, opts=opts)
    torch.cuda.synchronize()
    dt = _t.perf_counter() - t0
    steps = int(r["iters"][0])
    Pg = r["P"][0]
    log(f"point leg: {dt:.1f} s, {steps} steps, status {int(r['status'][0])}")
    return dict(seconds=round(dt, 3), solves_per_s=round(1.0 / dt, 4), status=int(r["status"][0]),
                steps=steps, ms_per_step=round(dt * 1e3 / max(1, steps), 4),
                H0=float(r["H0"][0]), Hmin=float(r["Hmin"][0]),
                y_mirror_max_diff=float((Pg - Pg.flip(1)).abs().max()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-ehl", action="store_true")
    ap.add_argument("--ehl-sweep", type=int, default=512,
                    help="instances of the line-contact sweep leg (N in {1025, 2049, 4097})")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-point", action="store_true")
    ap.add_argument("--rough-amp", type=float, default=0.005,
                    help="roughness amplitude of the adjoint leg")
    ap.add_argument("--point-n", type=int, default=257,
                    help="nodes per side of the point-contact leg")
    ap.add_argument("--sweep-cap64", action="store_true",
                    help="re-run the N=4097 sweep instances that stop on the active-set cap of 8 "
                         "with the default cap of 64 (about 80 s more)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a 256 MiB device copy (scale of the HBM byte counters)")
    ap.add_argument("--partitioned-only", action="store_true",
                    help="run only the partitioned long-system leg (one JSON object)")
    ap.add_argument("--no-partitioned", action="store_true")
    ap.add_argument("--no-active30", action="store_true",
                    help="skip the config-2 run at ~30%% active (keeps counter runs to one batch)")
    ap.add_argument("--part-case", default="",
                    help="n:q:r -- the partitioned leg on this one case only")
    ap.add_argument("--step-mode", choices=("many", "streams", "serial"), default="many",
                    help="how a step runs its three q batches: one paqif_solve_lcp_many call "
                         "(default), a call per batch on a stream each, or the calls one "
                         "after another on one stream")
    ap.add_argument("--deformation-only", action="store_true",
                    help="run only the MFMA deformation leg and print its figures")
    ap.add_argument("--convdiff-only", action="store_true",
                    help="run only the convection-diffusion leg (one JSON object)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on a single GPU; --gpus above 1 is not supported "
              "(batches shard by rows across GPUs with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2008_03276_amd as P

    if args.copy_calibration:
        # 2^25 doubles read and written once by torch's copy kernel
        src = torch.rand(1 << 25, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 8}))
        return
    P.lib()
    if args.deformation_only:
        print(json.dumps({"deformation_mfma": deformation_leg(P, torch, args)}))
        return
    if args.convdiff_only:
        print(json.dumps({"convdiff": convdiff_leg(P, torch, args)}))
        return
    if args.partitioned_only:
        print(json.dumps({"partitioned": partitioned_leg(P, torch, synth, args)}))
        return
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    batches = {}
    gpu = {}
    for q in QS:
        offs, band, f = synth.lcp_batch(COUNT, q, seed=args.seed)
        batches[q] = (offs, band, f)
        bt = P.paqif.Batch(offs, q, device=dev, order="lpt")
        gpu[q] = dict(bt=bt, band=torch.as_tensor(band, device=dev),
                      f=torch.as_tensor(f, device=dev),
                      ws64=bt.workspace(P.PREC_FP64), ws32=bt.workspace(P.PREC_FP32_IR))
    torch.cuda.synchronize()

    # the three q batches of a step are independent.  By default a step is
    # one paqif_solve_lcp_many call: every batch's start sweeps, then one
    # launch whose workgroups interleave the batches' waves (largest systems
    # first in each), so the batches share the chip from the start (measured
    # with about one active-set solve per LCP: 4.20-4.22 ms per step, against
    # 4.45 with a call per batch on a stream each and 5.5 one after another).
    # The FP32 + refinement leg has no row layout: its calls run on a stream
    # each.  The step ends when all its work has finished (the next waits).
    launch_order = sorted(QS, reverse=True)
    main_stream = torch.cuda.current_stream()
    step_mode = args.step_mode
    streams = {q: torch.cuda.Stream() for q in QS}

    step_ev = []  # HIP events on the main stream around each timed step

    def step(prec, ev=None):
        out = {}
        if ev is not None:
            s0 = torch.cuda.Event(enable_timing=True)
            s0.record(main_stream)
        ws = "ws64" if prec == P.PREC_FP64 else "ws32"
        if step_mode == "many" and prec == P.PREC_FP64:
            res = P.paqif.solve_lcp_many(
                [dict(batch=gpu[q]["bt"], band=gpu[q]["band"], b=gpu[q]["f"], workspace=gpu[q][ws])
                 for q in launch_order], mode=P.LCP_EXACT, prec=prec, refine_tol=1e-10)
            out = dict(zip(launch_order, res))
        else:
            conc = step_mode != "serial"
            if conc:
                for st_ in streams.values():
                    st_.wait_stream(main_stream)
            for q in launch_order:
                g = gpu[q]
                if conc:
                    torch.cuda.set_stream(streams[q])
                e0 = e1 = None
                if ev is not None:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                out[q] = P.paqif.solve_lcp(g["bt"], g["band"], g["f"], mode=P.LCP_EXACT,
                                           prec=prec, workspace=g[ws], refine_tol=1e-10)
                if ev is not None:
                    e1.record()
                    ev[q].append((e0, e1, out[q]))
                if conc:
                    torch.cuda.set_stream(main_stream)
            if conc:
                for st_ in streams.values():
                    main_stream.wait_stream(st_)
        if ev is not None:
            s1 = torch.cuda.Event(enable_timing=True)
            s1.record(main_stream)
            step_ev.append((prec, s0, s1, out))
        return out

    tune = {}
    for q in QS:
        g = gpu[q]
        for prec, ws in ((P.PREC_FP64, "ws64"), (P.PREC_FP32_IR, "ws32")):
            chosen, times = P.paqif.autotune(g["bt"], g["band"], g["f"], prec=prec,
                                             workspace=g[ws])
            tune[f"q{q}_{'fp64' if prec == P.PREC_FP64 else 'fp32ir'}"] = dict(
                layout=chosen, ms=[round(t, 3) for t in times],
                start_sweeps=P.paqif.get_start_sweeps(q, prec))
    log(f"autotuned layouts: {tune}")
    # the calls' start sweeps were tuned one batch at a time; the step runs
    # the three together, where fewer sweeps can pay (the chip is shared):
    # a coordinate search over the sweep counts, one q at a time, timing
    # whole steps (HIP events), keeps the fastest combination
    def step_ms_now(reps=5):
        for _ in range(2):
            step(P.PREC_FP64)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            step(P.PREC_FP64)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    best = {q: P.paqif.get_start_sweeps(q, P.PREC_FP64) for q in QS}
    best_ms = step_ms_now()
    tried = {",".join(str(best[q]) for q in QS): round(best_ms, 4)}
    for q in launch_order:
        for k in (8, 12, 16, 20, 24, 32):
            if k == best[q]:
                continue
            P.paqif.set_start_sweeps(q, P.PREC_FP64, k)
            ms = step_ms_now()
            tried[",".join(str(k if p_ == q else best[p_]) for p_ in QS)] = round(ms, 4)
            if ms < best_ms:
                best_ms, best[q] = ms, k
        P.paqif.set_start_sweeps(q, P.PREC_FP64, best[q])
    tune["step_start_sweeps"] = dict(chosen={str(q): best[q] for q in QS},
                                     step_ms=round(best_ms, 4), tried_q2_q4_q8=tried)
    log(f"start sweeps for the step: {best} ({best_ms:.3f} ms)")
    log("inputs resident; warm-up")
    for _ in range(args.warmup):
        step(P.PREC_FP64)
    torch.cuda.synchronize()
    log("timed LCP steps")

    # timed region: K steps (events around each step on the main stream; in
    # the stream and serial modes also around each call on its stream)
    ev = {q: [] for q in QS}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(P.PREC_FP64, ev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    solves_per_s = len(QS) * COUNT / (ms_per_step / 1e3)
    # each solve call alone on the GPU (after the timed region): the calls'
    # own durations for the standalone roofline
    alone = {q: [] for q in QS}
    for q in QS:
        g = gpu[q]
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            P.paqif.solve_lcp(g["bt"], g["band"], g["f"], mode=P.LCP_EXACT, prec=P.PREC_FP64,
                              workspace=g["ws64"])
            e1.record()
            alone[q].append((e0, e1))
    torch.cuda.synchronize()

    last = [o for p_, _, _, o in step_ev if p_ == P.PREC_FP64][-1]
    per_q = {}
    for q in QS:
        r = last[q]
        iters = r["iters"].cpu().numpy().astype(np.int64)
        status = r["status"].cpu().numpy()
        sizes = batches[q][0][1:] - batches[q][0][:-1]
        units = int((sizes * iters).sum())  # rows x active-set iterations
        sw = P.paqif.get_start_sweeps(q, P.PREC_FP64)
        bytes_sweeps = sweep_bytes(q, sizes, sw)
        bytes_alg = units * algorithmic_bytes_per_row(q) + bytes_sweeps
        alone_ms = float(np.mean([a.elapsed_time(b) for a, b in alone[q]]))
        # in the stream / serial modes: the call's own HIP events in the step
        in_step = ({"avg_ms": float(np.mean([a.elapsed_time(b) for a, b, _ in ev[q]]))}
                   if ev[q] else {})
        per_q[q] = dict(**in_step, alone_ms=alone_ms, iters_mean=float(iters.mean()),
                        iters_max=int(iters.max()), start_sweeps=sw,
                        sweep_bytes_gb=round(bytes_sweeps / 1e9, 4),
                        status_ok=bool((status == 0).all()),
                        kernel=lcp_call_kernels(P, q, P.PREC_FP64),
                        active_frac=float(r["active"].float().mean().item()),
                        gbs_alone=bytes_alg / (alone_ms / 1e3) / 1e9, bytes=bytes_alg)

    log(f"LCP fp64: {ms_per_step:.2f} ms/step")
    # mixed precision (FP32 factors + FP64 refinement to 1e-10): same
    # workload, HIP events per solve as above
    for _ in range(max(1, args.warmup // 2)):
        step(P.PREC_FP32_IR)
    torch.cuda.synchronize()
    evm = {q: [] for q in QS}
    tm0 = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        step(P.PREC_FP32_IR, evm)
    torch.cuda.synchronize()
    ms_mixed = (time.perf_counter() - tm0) * 1e3 / max(1, args.steps // 2)
    rm = {q: evm[q][-1][2] for q in QS}
    r64 = step(P.PREC_FP64)
    torch.cuda.synchronize()
    mixed_err = 0.0
    mixed_active_match = True
    per_q_mixed = {}
    for q in QS:
        u64 = r64[q]["u"]
        mixed_err = max(mixed_err, float((rm[q]["u"] - u64).abs().max() /
                                         max(1.0, float(u64.abs().max()))))
        mixed_active_match &= bool(torch.equal(rm[q]["active"], r64[q]["active"]))
        durs = [a.elapsed_time(b) for a, b, _ in evm[q]]
        st = rm[q]["status"].cpu().numpy()
        its = rm[q]["iters"].cpu().numpy().astype(np.int64)
        sizes = batches[q][0][1:] - batches[q][0][:-1]
        bytes_alg = int((sizes * its).sum()) * mixed_bytes_per_row(q) + \
            sweep_bytes(q, sizes, P.paqif.get_start_sweeps(q, P.PREC_FP32_IR))
        avg = float(np.mean(durs))
        per_q_mixed[q] = dict(avg_ms=round(avg, 4), iters_mean=round(float(its.mean()), 4),
                              statuses={str(int(k)): int(v)
                                        for k, v in zip(*np.unique(st, return_counts=True))},
                              gbs=round(bytes_alg / (avg / 1e3) / 1e9, 2),
                              kernel=lcp_call_kernels(P, q, P.PREC_FP32_IR), bytes=bytes_alg)
    domm = max(QS, key=lambda q: per_q_mixed[q]["avg_ms"])
    mixed_roof = dict(bound="hbm", achieved=per_q_mixed[domm]["gbs"], peak=HBM_PEAK_GBS,
                      unit="GB/s", frac=round(per_q_mixed[domm]["gbs"] / HBM_PEAK_GBS, 4),
                      traffic=None, kernel=per_q_mixed[domm]["kernel"],
                      algorithmic_bytes_per_launch_gb=round(per_q_mixed[domm]["bytes"] / 1e9, 3),
                      bytes_per_row_iteration=mixed_bytes_per_row(domm))

    active30 = active30_leg(P, torch, synth, args) if not args.no_active30 else None
    ehl = ehl_legs(P, torch, synth, dev, args) if not args.no_ehl else None
    deform = deformation_leg(P, torch, args) if not args.no_ehl else None
    part = partitioned_leg(P, torch, synth, args) if not args.no_partitioned else None
    copy_gbs = copy_bandwidth(torch)

    dom = max(QS, key=lambda q: per_q[q]["alone_ms"])
    step_ms = float(np.mean([a.elapsed_time(b) for p_, a, b, _ in step_ev
                             if p_ == P.PREC_FP64]))
    step_bytes = sum(per_q[q]["bytes"] for q in QS)
    step_gbs_ev = step_bytes / (step_ms / 1e3) / 1e9
    # the launch unit is the step: its three calls' algorithmic bytes over
    # its duration (HIP events on the main stream around it)
    if step_mode == "many":
        sweeps = [f"paqif_sweep_kernel<{q}>" for q in launch_order
                  if P.paqif.get_start_sweeps(q, P.PREC_FP64) > 0]
        kernel = ("step: " + " + ".join(sweeps) + (" then " if sweeps else "") +
                  "paqif_lcp_rows_many_kernel (q = " +
                  ", ".join(str(q) for q in launch_order) + " in one launch)")
        timing = ("HIP events on the main stream around each step: one "
                  "paqif_solve_lcp_many call (the three batches' start sweeps, then one "
                  "solve launch)")
        # the committed counter summary names the step's kernels joined by "+"
        tr_step = measured_step_traffic("+".join(
            [f"paqif_sweep_kernel<{q}>" for q in launch_order
             if P.paqif.get_start_sweeps(q, P.PREC_FP64) > 0] + ["paqif_lcp_rows_many_kernel"]))
    else:
        sep = " || " if step_mode == "streams" else " then "
        kernel = "step: " + sep.join(per_q[q]["kernel"] for q in launch_order) + (
            " (one stream per q)" if step_mode == "streams" else " (one stream)")
        timing = ("HIP events on the main stream around each step; its three q calls " +
                  ("run concurrently, one stream each" if step_mode == "streams"
                   else "one after another"))
        tr_step = None
    roof = dict(bound="hbm", achieved=round(step_gbs_ev, 2), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(step_gbs_ev / HBM_PEAK_GBS, 4),
                traffic=None if tr_step is None else round(tr_step / 1e9, 3),
                kernel=kernel, step_ms_events=round(step_ms, 4),
                algorithmic_bytes_per_launch_gb=round(step_bytes / 1e9, 3), timing=timing)
    # the same unit: without the start sweeps' bytes, and with only the band,
    # b and u reads
    ref_s = step_ms / 1e3
    no_sw = sum(per_q[q]["bytes"] - per_q[q]["sweep_bytes_gb"] * 1e9 for q in QS)
    min_b = sum((per_q[q]["bytes"] - per_q[q]["sweep_bytes_gb"] * 1e9) /
                algorithmic_bytes_per_row(q) * minimum_bytes_per_row(q) for q in QS)
    roof["frac_without_start_sweeps"] = round(no_sw / ref_s / 1e9 / HBM_PEAK_GBS, 4)
    roof["frac_minimum_bytes"] = round(min_b / ref_s / 1e9 / HBM_PEAK_GBS, 4)
    # the dominant call (the longest alone) on its own on the GPU, with the
    # counter traffic of that call when the summary holds it
    tr = measured_traffic(dom, per_q[dom]["kernel"].replace(" ", ""))
    roof["dominant_call_alone"] = dict(kernel=per_q[dom]["kernel"],
                                       ms=round(per_q[dom]["alone_ms"], 4),
                                       achieved=round(per_q[dom]["gbs_alone"], 2),
                                       frac=round(per_q[dom]["gbs_alone"] / HBM_PEAK_GBS, 4),
                                       algorithmic_bytes_per_launch_gb=round(
                                           per_q[dom]["bytes"] / 1e9, 3),
                                       traffic=None if tr is None else round(tr / 1e9, 3))
    roof["copy_kernel_gbs"] = round(copy_gbs, 1)
    roof["frac_vs_copy"] = round(roof["achieved"] / copy_gbs, 4)
    if roof["traffic"] is not None:
        roof["traffic_unit"] = "GB per step (FETCH_SIZE x2.0 + WRITE_SIZE, copy-calibrated)"
        roof["measured_hbm_gbs"] = round(roof["traffic"] / ref_s, 2)

    log(f"LCP mixed: {ms_mixed:.2f} ms/step")
    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        nthreads = os.cpu_count() or 1
        v = cpu_baseline(batches, args.cpu_sample, nthreads)
        cpu = dict(value=round(v, 2), unit="LCP solves/s", cores=nthreads, kind="oracle",
                   cpu_model=cpu_model(),
                   sample=(f"all {COUNT} systems of each q batch" if args.cpu_sample >= COUNT
                           else f"first {args.cpu_sample} systems of each q batch")
                          + ", exact LCP, OpenMP over systems",
                   build="C oracle, gcc -O3 -march=x86-64-v3 -ffp-contract=off -fopenmp",
                   ehl_oracle_note="the EHL oracle times in the ehl leg are numpy in one "
                                   "process (not threaded)")

    line = {
        "metric": "PAQIF banded-LCP solves/s (exact LCP, FP64)",
        "value": round(solves_per_s, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched banded LCP: 3 x 4096 systems, n~U[513,4097], "
                               "q in {2,4,8}, b~N(0,1)",
                   "systems_per_step": len(QS) * COUNT,
                   "q_batches": {"many": "one paqif_solve_lcp_many call",
                                 "streams": "concurrent, one stream each",
                                 "serial": "one after another"}[step_mode]},
        "per_q": {str(q): {k: (round(v, 4) if isinstance(v, float) else v)
                           for k, v in per_q[q].items() if k != "bytes"} for q in QS},
        "mixed_fp32_ir": {"ms_per_step": round(ms_mixed, 4),
                          "solves_per_s": round(len(QS) * COUNT / (ms_mixed / 1e3), 2),
                          "speedup_vs_fp64": round(ms_per_step / ms_mixed, 4),
                          "max_rel_err_vs_fp64": mixed_err,
                          "active_set_match": mixed_active_match,
                          "per_q": {str(q): {k: v for k, v in per_q_mixed[q].items()
                                             if k != "bytes"} for q in QS},
                          "roofline": mixed_roof},
        "autotune": tune,
        "ehl": ehl,
        "partitioned": part,
        "config2_active30": active30,
        "deformation_mfma": deform,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
