"""Write the oracle's converged EHL solutions at the sizes and parameters of
the line-contact sweep, the adjoint batch and the point contact, for the
GPU parity tests (tests/test_gpu_config_sizes.py).

Every stored value comes from ``oracle/`` (plain FP64 CPU code) on seeded
inputs from ``synth/``; nothing here touches the GPU library.  The oracle
needs minutes per instance at these sizes, so the results are computed once
and stored (NumPy .npz, loaded with allow_pickle=False).

    python tests/golden/make_ehl_configs.py [sweep|adjoint|point ...]
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# instances of the 512-instance sweep (M log-uniform in [10, 1000], L
# uniform in [5, 20], seed 0; groups of consecutive indices per N) compared
# with the oracle: two per N for N = 1025 and 2049, one for N = 4097
SWEEP_CASES = [(1025, 3), (1025, 5), (2049, 172), (2049, 180), (4097, 349)]
# first instances of the 64-instance adjoint batch (M log-uniform in
# [20, 500], L = 10, seed 0), roughness 0.005 sin(2 pi X / 0.25)
ADJ_N, ADJ_CASES, ADJ_AMP = 2049, [0, 1, 2], 0.005
# point contact at M = 200, L = 10 on a 65 x 65 grid of [-4.5, 1.5] x [-3, 3]
POINT_N, POINT_M, POINT_L = 65, 200.0, 10.0


def _sweep_case(case):
    import synth
    from oracle import ehl_line as OE
    N, i = case
    M, L = synth.ehl_sweep_params(512, seed=0)
    r = OE.solve_line(float(M[i]), float(L[i]), N, max_newton=3000, stall_steps=600)
    return dict(N=N, index=i, M=float(M[i]), L=float(L[i]), P=r["P"], H=r["H"], H0=r["H0"],
                Hmin=r["Hmin"], status=r["status"], iters=r["iters"])


def _adjoint_case(i):
    import synth
    from oracle import ehl_adjoint as OA
    from oracle import ehl_line as OE
    M, L = synth.ehl_adjoint_params(64, seed=0)
    x, _ = OE.grid(ADJ_N)
    rough = synth.roughness(x, amplitude=ADJ_AMP)
    r = OE.solve_line(float(M[i]), float(L[i]), ADJ_N, rough=rough)
    out = dict(index=i, M=float(M[i]), L=float(L[i]), P=r["P"], H=r["H"], H0=r["H0"],
               Hmin=r["Hmin"], status=r["status"], iters=r["iters"])
    if r["status"] == 0:
        g = OA.adjoint_gradients(r["P"], r["H0"], float(M[i]), float(L[i]), ADJ_N, rough=rough)
        for k in ("dH0_dM", "dH0_dL", "dHmin_dM", "dHmin_dL", "dH0_drough", "dHmin_drough",
                  "argmin"):
            out[k] = g[k]
    return out


def _point_case(_):
    from oracle import ehl_point as OP
    r = OP.solve_point(POINT_M, POINT_L, POINT_N, POINT_N, tol=1e-13, max_steps=20000)
    return dict(P=r["P"], H=r["H"], H0=r["H0"], Hmin=r["Hmin"], status=r["status"],
                iters=r["iters"])


def _stack(results, keys):
    return {k: np.array([r[k] for r in results]) for k in keys}


def main(which):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    jobs = {}
    with ProcessPoolExecutor(max_workers=7) as ex:
        if "sweep" in which:
            jobs["sweep"] = [ex.submit(_sweep_case, c) for c in SWEEP_CASES]
        if "adjoint" in which:
            jobs["adjoint"] = [ex.submit(_adjoint_case, i) for i in ADJ_CASES]
        if "point" in which:
            jobs["point"] = [ex.submit(_point_case, 0)]
        for name, futs in jobs.items():
            res = [f.result() for f in futs]
            path = os.path.join(HERE, f"ehl_{name}_oracle.npz")
            if name == "sweep":
                arrs = {}
                for r in res:
                    tag = f"N{r['N']}_i{r['index']}"
                    for k in ("P", "H", "H0", "Hmin", "status", "iters", "M", "L"):
                        arrs[f"{tag}_{k}"] = np.asarray(r[k])
                np.savez_compressed(path, **arrs)
            elif name == "adjoint":
                arrs = {}
                for r in res:
                    tag = f"i{r['index']}"
                    for k, v in r.items():
                        if k != "index":
                            arrs[f"{tag}_{k}"] = np.asarray(v)
                np.savez_compressed(path, **arrs)
            else:
                np.savez_compressed(path, **{k: np.asarray(v) for k, v in res[0].items()})
            print(name, [(r.get("N"), r.get("index"), int(r["status"]), int(r["iters"]))
                         for r in res], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["sweep", "adjoint", "point"])
