"""The C-ABI library loads and exports every entry point that include/mihs.h
declares (no GPU calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mihs.h")
LIB = os.path.join(ROOT, "paper_1912_03514_amd", "libmihs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mihs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mihs_sketch", "mihs_solve", "mihs_solve_batched", "mihs_solve_backward",
                     "mihs_create", "mihs_destroy", "mihs_status_string"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmihs.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for name in declared_functions():
        assert name in exported, name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmihs.so not built")
def test_binding_signatures_cover_header():
    import paper_1912_03514_amd as mihs
    assert set(declared_functions()) == set(mihs.EXPORTED)
    lib = mihs.load_library()
    assert lib.mihs_status_string(-1) == b"invalid argument"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmihs.so not built")
def test_argument_validation_without_gpu():
    """Null handle and bad sizes are rejected on the host before any GPU call."""
    import paper_1912_03514_amd as mihs
    lib = mihs.load_library()
    sz = ctypes.c_size_t()
    assert lib.mihs_sketch_workspace_size(None, 10, 4, 4, 0, 0, 0, 0, ctypes.byref(sz)) == -1
    assert lib.mihs_solve(None, None, 0, 10, 4, 4, None, 1.0, None, 4, 4, 0, 0.5, 0.2, 1e-2,
                          1e-10, 10, 10, None, None, None, None, 0, None) == -1
    assert lib.mihs_destroy(None) == 0
