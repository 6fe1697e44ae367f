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
    return sorted(set(re.findall(r"\b(mihs_[a-z0-9_]+)\s*\(", text)))


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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmihs.so not built")
def test_momentum_entry_points_match_the_oracle():
    """mihs_momentum_cor4 / mihs_momentum_thm1 (host computations behind the
    C ABI) against the oracle's Corollary 4 and Theorem 1, whose own pins are
    Theorem 1's identity, its minimax characterisation and Figure 2's number."""
    import math
    import paper_1912_03514_amd as mihs
    from oracle import solver as O
    for sd, m in ((64, 256), (512, 2048), (1024, 4096), (1, 3), (999, 1000), (0.5, 7)):
        a, b = mihs.momentum(sd, m)
        ra, rb = O.momentum_cor4(sd, m)
        assert abs(a - ra) <= 1e-15 and abs(b - rb) <= 1e-15
    for eps in (1e-6, 0.1, 0.5, 0.9, 0.999):
        a, b = mihs.momentum_thm1(eps)
        ra, rb = O.momentum_thm1(eps)
        assert abs(a - ra) <= 1e-14 * max(1.0, ra) and abs(b - rb) <= 1e-14
    lib = mihs.load_library()
    x, y = ctypes.c_double(), ctypes.c_double()
    for sd, m in ((0.0, 10), (10.0, 10), (11.0, 10), (-1.0, 10), (float("nan"), 10), (1.0, 0)):
        assert lib.mihs_momentum_cor4(sd, m, ctypes.byref(x), ctypes.byref(y)) == -1
    for eps in (0.0, 1.0, -0.5, float("nan")):
        assert lib.mihs_momentum_thm1(eps, ctypes.byref(x), ctypes.byref(y)) == -1
    assert lib.mihs_momentum_cor4(1.0, 4, None, ctypes.byref(y)) == -1
    for ll in (-20.0, -3.9, 0.0, 2.5):
        assert mihs.lambda_from_log(ll) == math.exp(ll)
    assert lib.mihs_lambda_from_log(800.0, ctypes.byref(x)) == -1
    assert lib.mihs_lambda_from_log(-800.0, ctypes.byref(x)) == -1
