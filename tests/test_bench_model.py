"""The benchmark's algorithmic byte model (the roofline's numerator), on the
host: per-row bytes of an active-set iteration and of the start sweeps, with
the sweep launches split as the library splits them (at most 1 + 128/q
sweeps per launch)."""
import importlib.util
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_model", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_row_iteration_bytes():
    b = _bench()
    # band (2q+1 doubles) + b + u read, Z0 rows (2q+1 doubles) written and read
    assert [b.algorithmic_bytes_per_row(q) for q in (2, 4, 8)] == [136, 232, 424]
    assert [b.minimum_bytes_per_row(q) for q in (2, 4, 8)] == [56, 88, 152]
    # FP32 + refinement: FP64 band, b, u; FP32 Z (2q+3 per row) and W (2q per
    # row) records written and read (the FP64 kernel keeps no W: its forward
    # solve is fused into the factorisation)
    assert [b.mixed_bytes_per_row(q) for q in (2, 4, 8)] == [144, 240, 432]


def test_sweep_bytes_follow_the_launch_split():
    b = _bench()
    sizes = np.array([513, 4097, 1000])
    rows = int(sizes.sum())
    assert b.sweep_bytes(8, sizes, 0) == 0
    for q in (2, 4, 8):
        per_launch = 8 * (2 * q + 1) + 16  # band, b, iterate written
        kp = 1 + 128 // q
        for k in (1, kp, kp + 1, 32):
            launches = -(-k // kp)
            want = rows * (launches * per_launch + (launches - 1) * 8)
            assert b.sweep_bytes(q, sizes, k) == want, (q, k)
    # q = 8: 12 sweeps in one launch, 20 in two (17 at most per launch)
    assert b.sweep_bytes(8, sizes, 12) == rows * (8 * 17 + 16)
    assert b.sweep_bytes(8, sizes, 20) == rows * (2 * (8 * 17 + 16) + 8)
