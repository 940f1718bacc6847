"""The allocation-free LCP entry point (paqif_solve_lcp_noalloc) against the
workspace entry point (paqif_solve_lcp), through the C ABI.

Both run the same kernels on the same inputs; only where the level records,
active flags and refinement residual live differs (the library's own device
array instead of a caller workspace), so every output must agree bit for bit.
Two calls in a row, the second with a smaller batch, check that nothing left
in the shared array by the first call leaks into the second.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _inputs(q, sizes, seed):
    offs, band, f = synth.lcp_batch(len(sizes), q, seed=seed, sizes=sizes)
    dev = torch.device("cuda")
    return offs, torch.as_tensor(band, device=dev), torch.as_tensor(f, device=dev)


def _both(P, q, sizes, seed, mode, prec):
    offs, band, f = _inputs(q, sizes, seed)
    bt = P.paqif.Batch(offs, q, order="lpt")
    ref = P.paqif.solve_lcp(bt, band, f, mode=mode, prec=prec)
    dev = band.device
    rows = bt.total_rows
    out = dict(u=torch.full((rows,), np.nan, dtype=torch.float64, device=dev),
               w=torch.full((rows,), np.nan, dtype=torch.float64, device=dev),
               active=torch.full((rows,), 7, dtype=torch.uint8, device=dev),
               status=torch.full((bt.count,), -9, dtype=torch.int32, device=dev),
               iters=torch.full((bt.count,), -9, dtype=torch.int32, device=dev))
    code = P.paqif.solve_lcp_noalloc(bt, band, f, out["u"], out["status"], mode=mode, prec=prec,
                                     w=out["w"], active=out["active"], iters=out["iters"])
    torch.cuda.synchronize()
    assert code == 0, code
    return ({k: v.cpu().numpy() for k, v in ref.items()},
            {k: v.cpu().numpy() for k, v in out.items()})


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("q", [2, 4, 8])
def test_noalloc_matches_workspace_entry_two_calls(gpu, q, prec):
    first = [4097, 3000, 2049, 1025, 777, 513, 64, 9, 2, 1]
    second = [1500, 700, 100, 33, 5]  # smaller: fewer systems and rows
    for sizes, seed in ((first, 40 + q), (second, 50 + q)):
        ref, got = _both(gpu, q, sizes, seed, mode=2, prec=prec)
        assert (ref["status"] == 0).all(), ref["status"]
        for k in ("u", "w", "active", "status", "iters"):
            assert np.array_equal(ref[k], got[k]), k


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_linear_and_clip(gpu, mode):
    ref, got = _both(gpu, 4, [300, 41, 8], 61, mode=mode, prec=0)
    for k in ("u", "w", "active", "status", "iters"):
        assert np.array_equal(ref[k], got[k]), k


def test_noalloc_refuses_a_batch_beyond_its_scratch(gpu):
    P = gpu
    # q = 8, FP64: 152 bytes per row of records; 600 systems of 4097 rows
    # need about 375 MB, beyond the 64 MiB array: refused on the host
    sizes = [4097] * 600
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    bt = P.paqif.Batch(offs, 8)
    dev = torch.device("cuda")
    rows = bt.total_rows
    band = torch.zeros(rows * 17, dtype=torch.float64, device=dev)
    f = torch.zeros(rows, dtype=torch.float64, device=dev)
    u = torch.zeros(rows, dtype=torch.float64, device=dev)
    st = torch.full((bt.count,), -9, dtype=torch.int32, device=dev)
    code = P.paqif.solve_lcp_noalloc(bt, band, f, u, st, mode=2)
    torch.cuda.synchronize()
    assert code == P._binding.PAQIF_EWORKSPACE
    assert (st.cpu().numpy() == -9).all()  # nothing was launched
