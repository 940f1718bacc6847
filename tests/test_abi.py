"""The C-ABI library loads on the CPU host and exports every entry point the
public header declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for f in os.listdir(os.path.join(ROOT, "include")):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(",
                             text, flags=re.M):
            if not m.group(0).lstrip().startswith(("typedef", "#")):
                names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["paqif_factor", "paqif_solve_lcp", "ehl_deformation",
                     "ehl_jacobian_assemble", "ehl_newton_tvd"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2008_03276_amd import _binding
    path = _binding.library_path()
    if not os.path.exists(path):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_2008_03276_amd import _binding
    if not os.path.exists(_binding.library_path()):
        pytest.skip("library not built")
    L = _binding.lib()
    for n in declared_functions():
        assert getattr(L, n).argtypes is not None, n


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2008_03276_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f
