"""Partitioned PAQIF (one long band system over r blocks) on the GPU vs the
FP64 oracle, same seeded inputs, element by element.

Tolerance: the GPU eliminates each block's inner unknowns with the batched
PAQIF kernel and forms the reduced system as a Schur complement, where the
oracle uses dense W0/Z0 factors and the W0-scaled reduced rows; both are
FP64 on strictly diagonally dominant systems (condition numbers below ~50),
so the results differ by rounding order only: 1e-11 relative.
  * small cases (ragged splits, odd/even blocks, one block, minimum blocks
    of 2q+1 rows, q = 2 cases whose reduced system is partitioned again) in
    linear and clip mode, all rows or a mask bounded;
  * mid-size cases against the oracle's monolithic AQIF solve (linear) and
    the oracle's partitioned solve (clip);
  * the benchmark's size (n = 2^20, q = 2, r = 512, linear) against the
    oracle's monolithic AQIF solve in full;
  * exact mode (the LCP of eq. 14 by an active-set iteration around the
    partitioned solve): u within 1e-11 of the oracle's exact LCP solver and
    the same active set, element by element (the solution of an LCP with a
    strictly diagonally dominant matrix is unique), small to n = 2^20;
  * argument checks.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import partitioned as OP

pytestmark = pytest.mark.gpu

CASES = [(60, 2, 4), (61, 2, 4), (97, 2, 7), (50, 2, 1), (35, 2, 7), (200, 4, 6), (203, 4, 5),
         (72, 4, 8), (1000, 2, 33), (1001, 4, 21),
         # q = 2 with at least 512 reduced rows: the reduced system is partitioned again
         (3000, 2, 128), (2601, 2, 131)]


def _gpu(P, band, f, r, mode, bounded=None, full=False):
    dev = torch.device("cuda")
    bnd = None if bounded is None else torch.as_tensor(bounded, dtype=torch.uint8, device=dev)
    res = P.paqif.solve_partitioned(torch.as_tensor(band, device=dev),
                                    torch.as_tensor(f, device=dev), r, mode=mode, bounded=bnd)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in res.items()}
    if full:
        return out
    return out["u"], int(out["status"][0])


def _rel(a, b):
    return np.abs(a - b).max() / max(1.0, np.abs(b).max())


@pytest.mark.parametrize("N,q,r", CASES)
@pytest.mark.parametrize("mode", [oracle.LINEAR, oracle.CLIP])
@pytest.mark.parametrize("masked", [False, True])
def test_parity_small(gpu, N, q, r, mode, masked):
    print(f"partitioned N={N} q={q} r={r} mode={mode} masked={masked}", flush=True)
    band, f = synth.long_system(N, q, seed=N + r)
    bounded = None
    if masked:
        bounded = (np.random.default_rng(N).random(N) < 0.7).astype(np.uint8)
    u, st = _gpu(gpu, band, f, r, mode, bounded)
    assert st == 0
    ref = OP.solve_partitioned(band, f, r, bounded=bounded, mode=mode)
    assert _rel(u, ref) <= 1e-11


@pytest.mark.parametrize("N,q,r", [(20000, 2, 64), (20000, 2, 256), (20011, 4, 40)])
def test_parity_mid(gpu, N, q, r):
    print(f"partitioned mid N={N} q={q} r={r}", flush=True)
    band, f = synth.long_system(N, q, seed=11)
    u, st = _gpu(gpu, band, f, r, oracle.LINEAR)
    assert st == 0
    ref, ost = oracle.aqif_solve(band, f)
    assert ost == 0
    assert _rel(u, ref) <= 1e-11
    u, st = _gpu(gpu, band, f, r, oracle.CLIP)
    assert st == 0
    ref = OP.solve_partitioned(band, f, r, mode=oracle.CLIP)
    assert _rel(u, ref) <= 1e-11
    assert (u >= 0).all()


def test_parity_bench_size(gpu):
    N, q, r = 1 << 20, 2, 512
    print(f"partitioned full N={N} q={q} r={r}", flush=True)
    band, f = synth.long_system(N, q, seed=0)
    u, st = _gpu(gpu, band, f, r, oracle.LINEAR)
    assert st == 0
    ref, ost = oracle.aqif_solve(band, f)
    assert ost == 0
    assert _rel(u, ref) <= 1e-11


EXACT_CASES = [(60, 2, 4), (97, 2, 7), (50, 2, 1), (200, 4, 6), (1001, 4, 21), (3000, 2, 128),
               (20000, 2, 256), (20011, 4, 40)]


@pytest.mark.parametrize("N,q,r", EXACT_CASES)
@pytest.mark.parametrize("masked", [False, True])
def test_exact_matches_oracle_lcp(gpu, N, q, r, masked):
    print(f"partitioned exact N={N} q={q} r={r} masked={masked}", flush=True)
    band, f = synth.long_system(N, q, seed=3 * N + r)
    bounded = None
    if masked:
        bounded = (np.random.default_rng(N + 1).random(N) < 0.7).astype(np.uint8)
    g = _gpu(gpu, band, f, r, oracle.EXACT, bounded, full=True)
    assert int(g["status"][0]) == 0
    o = oracle.lcp_solve(band, f, bounded=bounded, mode=oracle.EXACT, max_iter=64)
    assert o["status"] == 0
    assert _rel(g["u"], o["u"]) <= 1e-11
    assert np.array_equal(g["active"], o["active"])
    assert 1 <= int(g["iters"][0]) <= 64


def test_exact_bench_size(gpu):
    N, q, r = 1 << 20, 2, 2048
    print(f"partitioned exact full N={N} q={q} r={r}", flush=True)
    band, f = synth.long_system(N, q, seed=5)
    g = _gpu(gpu, band, f, r, oracle.EXACT, full=True)
    assert int(g["status"][0]) == 0
    o = oracle.lcp_solve(band, f, mode=oracle.EXACT, max_iter=64)
    assert o["status"] == 0
    assert _rel(g["u"], o["u"]) <= 1e-11
    assert np.array_equal(g["active"], o["active"])


def test_exact_not_converged_status(gpu):
    # one active-set solve is not enough from A_0 here: status says so
    band, f = synth.long_system(2000, 2, seed=9)
    dev = torch.device("cuda")
    res = gpu.paqif.solve_partitioned(torch.as_tensor(band, device=dev),
                                      torch.as_tensor(f, device=dev), 16, mode=oracle.EXACT,
                                      max_iter=1)
    torch.cuda.synchronize()
    assert int(res["status"].cpu()[0]) == oracle.LCP_NOT_CONVERGED
    assert int(res["iters"].cpu()[0]) == 1


def test_invalid_arguments(gpu):
    band, f = synth.long_system(100, 2, seed=1)
    for r, mode in ((0, 0), (21, 0), (4, 7)):      # r = 21: blocks of 4 < 2q+1 rows; mode 7
        with pytest.raises(RuntimeError):
            _gpu(gpu, band, f, r, mode)
    dev = torch.device("cuda")
    with pytest.raises(RuntimeError):
        gpu.paqif.solve_partitioned(torch.as_tensor(band, device=dev),
                                    torch.as_tensor(f, device=dev), 4, mode=oracle.EXACT,
                                    max_iter=0)
    band8, f8 = synth.long_system(200, 8, seed=1)            # q = 8: reduced band 16 unsupported
    with pytest.raises(RuntimeError):
        _gpu(gpu, band8, f8, 4, oracle.LINEAR)
    assert gpu.paqif.partitioned_workspace_bytes(100, 2, 21) == 0
    assert gpu.paqif.partitioned_workspace_bytes(100, 2, 20) > 0


def test_graph_replay_matches_eager(gpu):
    # linear and clip modes launch kernels only (no host synchronisation, no
    # memset), so the solve can be captured; every replay, with other work
    # between replays, must give the eager result bit for bit
    N, q, r = 20000, 2, 256
    band_h, f_h = synth.long_system(N, q, seed=21)
    dev = torch.device("cuda")
    band = torch.as_tensor(band_h, device=dev)
    f = torch.as_tensor(f_h, device=dev)
    ws = torch.empty(gpu.paqif.partitioned_workspace_bytes(N, q, r), dtype=torch.uint8, device=dev)
    for mode in (oracle.LINEAR, oracle.CLIP):
        eager = gpu.paqif.solve_partitioned(band, f, r, mode=mode, workspace=ws)["u"].clone()
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            gpu.paqif.solve_partitioned(band, f, r, mode=mode, workspace=ws)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            out = gpu.paqif.solve_partitioned(band, f, r, mode=mode, workspace=ws)
        for k in range(3):
            junk = torch.randn(1 << 16, device=dev).sum()   # eager work between replays
            torch.cuda.synchronize()
            out["u"].zero_()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out["u"], eager), (mode, k)
            assert int(out["status"].cpu()[0]) == 0
            del junk
