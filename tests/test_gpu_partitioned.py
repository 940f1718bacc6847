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


def _gpu(P, band, f, r, mode, bounded=None):
    dev = torch.device("cuda")
    bnd = None if bounded is None else torch.as_tensor(bounded, dtype=torch.uint8, device=dev)
    u, st = P.paqif.solve_partitioned(torch.as_tensor(band, device=dev),
                                      torch.as_tensor(f, device=dev), r, mode=mode, bounded=bnd)
    torch.cuda.synchronize()
    return u.cpu().numpy(), int(st.cpu()[0])


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


def test_invalid_arguments(gpu):
    band, f = synth.long_system(100, 2, seed=1)
    for r, mode in ((0, 0), (21, 0), (4, oracle.EXACT)):      # r = 21: blocks of 4 < 2q+1 rows
        with pytest.raises(RuntimeError):
            _gpu(gpu, band, f, r, mode)
    band8, f8 = synth.long_system(200, 8, seed=1)            # q = 8: reduced band 16 unsupported
    with pytest.raises(RuntimeError):
        _gpu(gpu, band8, f8, 4, oracle.LINEAR)
    assert gpu.paqif.partitioned_workspace_bytes(100, 2, 21) == 0
    assert gpu.paqif.partitioned_workspace_bytes(100, 2, 20) > 0
