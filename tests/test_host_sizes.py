"""Host-side argument checks and workspace sizes of the C-ABI (pure host
code: the size queries touch no device, so they run on the CPU host).

  * the partitioned solve refuses q outside {2, 4}, r < 1, blocks of fewer
    than 2q+1 rows and n above 2^31 (size 0), and otherwise needs at least
    the right-hand sides, solutions and level records of its (2q+1) r block
    systems, growing with n;
  * for q = 2 a reduced system of at least 512 rows brings the workspace of
    its own partitioned solve (the size jumps where 2 q r reaches 512);
  * the convection-diffusion workspaces exist for 5 <= n <= 16385 only.
"""
import ctypes
import os

import pytest

from paper_2008_03276_amd import _binding


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_binding.library_path()):
        pytest.skip("library not built (run __graft_entry__.build())")
    return _binding.lib()


def test_partitioned_workspace_refusals(lib):
    f = lib.paqif_partitioned_workspace_bytes
    assert f(1000, 8, 10) == 0          # reduced band 16: unsupported
    assert f(1000, 3, 10) == 0
    assert f(1000, 2, 0) == 0
    assert f(1000, 2, 201) == 0         # blocks of 4 < 2q+1 rows
    assert f(1000, 2, 200) > 0          # blocks of 5 = 2q+1 rows
    assert f(1000, 4, 112) == 0         # blocks of 8 < 9 rows
    assert f((1 << 31) + 1, 2, 1024) == 0
    assert f(0, 2, 1) == 0


@pytest.mark.parametrize("q", [2, 4])
def test_partitioned_workspace_covers_the_block_solves(lib, q):
    f = lib.paqif_partitioned_workspace_bytes
    r = 16
    for n in (1000, 10000, 100000):
        W = 2 * q + 1
        Ni = n - 2 * q * r
        rows = W * Ni
        # rhs + solution (8 B each) and one level record (>= 4q+6 doubles)
        # per two rows of every block system
        assert f(n, q, r) >= rows * 16 + (rows // 2) * (4 * q + 6) * 8
    assert f(10000, q, r) < f(100000, q, r)


def test_nested_reduced_solve_adds_its_workspace(lib):
    f = lib.paqif_partitioned_workspace_bytes
    n = 1 << 16
    # q = 2: 2 q r = 508 reduced rows (solved whole) vs 512 (partitioned again)
    below, at = f(n, 2, 127), f(n, 2, 128)
    assert below > 0 and at > 0
    step_without_nesting = f(n, 2, 126) - f(n, 2, 127)
    assert at - below > abs(step_without_nesting)


def test_convdiff_workspaces(lib):
    for g in (lib.cd_workspace_bytes, lib.cd_ls3_workspace_bytes):
        assert g(4) == 0 and g(16386) == 0
        assert g(5) > 0 and g(257) > g(65) > 0
    # the Ls3 band has half-bandwidth 4 (9 entries per row) instead of 2
    assert lib.cd_ls3_workspace_bytes(257) > lib.cd_workspace_bytes(257)
