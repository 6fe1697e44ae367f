"""The gradient pass's row split over workgroups (mihs_row_split, host only):
equal weights give the even split floor(n v / G); other weights give shares
in proportion to the weight of each workgroup's XCD (workgroup v on XCD v mod 8);
the bounds always run from 0 to n without decreasing."""
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1912_03514_amd", "libmihs.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmihs.so not built")


def _split(n, G, w):
    import paper_1912_03514_amd as mihs
    return mihs.row_split(n, G, w)


@pytest.mark.parametrize("n,G", [(262144, 256), (1 << 20, 512), (4096, 64), (1000, 13),
                                 (5, 8), (0, 4), (7, 1)])
def test_equal_weights_give_the_even_split(n, G):
    for w in ([64] * 8, [1] * 8, [37] * 8):
        assert _split(n, G, w) == [n * v // G for v in range(G + 1)]


@pytest.mark.parametrize("n,G", [(262144, 256), (100003, 100), (1 << 20, 512), (300, 256)])
@pytest.mark.parametrize("w", [[64, 60] * 4, [64, 32, 48, 63, 40, 64, 33, 50], [1, 64] * 4])
def test_weighted_shares_follow_the_xcd_weights(n, G, w):
    b = _split(n, G, w)
    assert b[0] == 0 and b[-1] == n
    assert all(b[v] <= b[v + 1] for v in range(G))
    # P(v) = sum of w[u mod 8] over u < v; bound(v) = floor(n P(v) / P(G))
    P = [0]
    for v in range(G):
        P.append(P[-1] + w[v % 8])
    assert b == [n * P[v] // P[G] for v in range(G)] + [n]
    # each share is within one row of its exact proportion
    for v in range(G):
        exact = n * w[v % 8] / P[G]
        assert abs((b[v + 1] - b[v]) - exact) < 1.0 + 1e-9


def test_invalid_arguments_are_rejected():
    import ctypes
    import paper_1912_03514_amd as mihs
    lib = mihs.load_library()
    W8 = ctypes.c_int32 * 8
    out = (ctypes.c_int64 * 9)()
    assert lib.mihs_row_split(100, 8, W8(*([64] * 7 + [0])), out) == -1
    assert lib.mihs_row_split(100, 8, W8(*([64] * 7 + [65])), out) == -1
    assert lib.mihs_row_split(-1, 8, W8(*([64] * 8)), out) == -1
    assert lib.mihs_row_split(100, 0, W8(*([64] * 8)), out) == -1
    assert lib.mihs_set_row_weights(None, None) == -1
    assert lib.mihs_get_row_weights(None, W8()) == -1
    assert lib.mihs_calibrate_rows(None, None) == -1
