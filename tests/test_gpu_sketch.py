"""GPU parity: the sketch kernels against the oracle's sketches."""
import math

import numpy as np
import pytest

from oracle import hashes, sketches
from gpu_common import announce, rel, requires_gpu, to_dev, torch

pytestmark = [pytest.mark.gpu, requires_gpu]


def _mihs():
    import paper_1912_03514_amd as mihs
    return mihs


def _rand(n, d, seed, dtype=np.float64):
    return np.random.default_rng(seed).standard_normal((n, d)).astype(dtype)


@pytest.mark.parametrize("n,d,m", [(64, 5, 16), (512, 33, 100), (4096, 70, 256),
                                   (1 << 14, 100, 300), (1 << 15, 17, 2048)])
def test_srht_plain(n, d, m):
    mihs = _mihs()
    A = _rand(n, d, n + d)
    ref = sketches.srht_sketch(A, m, 31)
    announce(f"srht plain n={n} d={d} m={m}")
    SA = mihs.mihs_sketch(to_dev(A), "srht", m, 31).cpu().numpy()
    # the GPU sums the transform in a different order: error ~ log2(n) ulps of sum |A|
    bound = 4 * math.log2(n) * 2.0 ** -52 * np.abs(A).sum(axis=0).max() / math.sqrt(m)
    assert np.max(np.abs(SA - ref)) <= bound


def test_srht_signs_and_samples_exact():
    """With A = I every entry of SA is +-1/sqrt(m) at the sampled Hadamard row
    times the sign diagonal: signs and sampled indices must match exactly."""
    mihs = _mihs()
    n, m = 1 << 12, 64
    A = np.eye(n)[:, :512].copy()
    announce("srht identity exactness")
    SA = mihs.mihs_sketch(to_dev(A), "srht", m, 77).cpu().numpy()
    D = sketches.srht_signs(n, 77)
    rows = sketches.srht_rows(m, n, 77)
    expect = sketches.hadamard_entry(rows[:, None], np.arange(512)[None, :]) * D[None, :512]
    assert np.array_equal(np.sign(SA), expect)
    assert np.allclose(np.abs(SA), 1 / math.sqrt(m), rtol=1e-15, atol=0)


@pytest.mark.parametrize("prec", ["plain", "mixed"])
def test_srht_full_size_whole_rows(prec):
    """At the headline size (2^18 x 2048 FP64, m = 2048) 16 whole sampled output
    rows (all 2048 columns) equal the direct O(n) sum of the definition; the
    bound is a few rounding errors of the partial sums (log2(n) levels) in the
    arithmetic's precision (FP64 plain, FP32 mixed)."""
    mihs = _mihs()
    n, d, m, seed = 1 << 18, 2048, 2048, 8
    g = torch.Generator(device="cuda").manual_seed(5)
    A = torch.randn(n, d, generator=g, dtype=torch.float64, device="cuda")
    announce(f"srht full size 2^18 x 2048 ({prec})")
    SA = mihs.mihs_sketch(A, "srht", m, seed, precision=prec).double().cpu().numpy()
    Ah = A.cpu().numpy()
    del A
    u = 2.0 ** -52 if prec == "plain" else 2.0 ** -23
    colsum = np.abs(Ah).sum(axis=0) / math.sqrt(m)
    rng = np.random.default_rng(0)
    ks = np.sort(rng.choice(m, 16, replace=False))
    for k in ks:
        ref = sketches.srht_entry(Ah, m, seed, int(k), slice(None))
        err = np.abs(SA[k] - ref)
        assert np.all(err <= 4 * math.log2(n) * u * colsum), (k, float(err.max()))


@pytest.mark.parametrize("prec", ["plain", "mixed"])
def test_srht_two_stage_above_2048_samples(prec):
    """More than 2048 sampled rows (ragged m = 3000) take the two-stage form: the
    blocked transform H D A over 512-row blocks written out, then the sampled
    rows combined across blocks.  Every entry is within a few rounding errors of
    the oracle's transform (log2(n) levels, in FP64 or FP32)."""
    mihs = _mihs()
    n, d, m = 1 << 14, 40, 3000
    A = _rand(n, d, 19)
    ref = sketches.srht_sketch(A, m, 23)
    announce(f"srht two-stage n={n} d={d} m={m} ({prec})")
    SA = mihs.mihs_sketch(to_dev(A), "srht", m, 23, precision=prec).double().cpu().numpy()
    assert SA.shape == (m, d)
    u = 2.0 ** -52 if prec == "plain" else 2.0 ** -23
    bound = 4 * math.log2(n) * u * np.abs(A).sum(axis=0).max() / math.sqrt(m)
    assert np.max(np.abs(SA - ref)) <= bound


@pytest.mark.parametrize("adt", [np.float64, np.float32])
def test_srht_mixed(adt):
    mihs = _mihs()
    n, d, m = 1 << 13, 50, 128
    A = _rand(n, d, 3, adt)
    ref = sketches.srht_sketch(A, m, 5)
    announce(f"srht mixed {adt.__name__}")
    SA = mihs.mihs_sketch(to_dev(A), "srht", m, 5, precision="mixed")
    assert SA.dtype == torch.float32
    SA = SA.cpu().numpy().astype(np.float64)
    bound = 4 * math.log2(n) * 2.0 ** -23 * np.abs(A).astype(np.float64).sum(axis=0).max() / math.sqrt(m)
    assert np.max(np.abs(SA - ref)) <= bound


@pytest.mark.parametrize("n,d,m", [(1, 3, 4), (300, 7, 16), (5000, 70, 128), (20000, 300, 1000),
                                   (70000, 33, 8192)])
def test_countsketch_bit_exact(n, d, m):
    """Rows are summed per bucket in ascending row order in FP64 on both sides:
    the result is bit-identical, which pins hashes, buckets and signs exactly."""
    mihs = _mihs()
    A = _rand(n, d, n)
    ref = sketches.countsketch(A, m, 12345)
    announce(f"countsketch n={n} d={d} m={m}")
    SA = mihs.mihs_sketch(to_dev(A), "countsketch", m, 12345).cpu().numpy()
    assert np.array_equal(SA, ref)


def test_countsketch_fp32_matrix():
    mihs = _mihs()
    A = _rand(10000, 64, 2, np.float32)
    ref = sketches.countsketch(A, 256, 9)
    announce("countsketch fp32 A plain")
    SA = mihs.mihs_sketch(to_dev(A), "countsketch", 256, 9).cpu().numpy()
    assert np.array_equal(SA, ref)  # float -> double is exact; same order
    announce("countsketch fp32 A mixed")
    SAm = mihs.mihs_sketch(to_dev(A), "countsketch", 256, 9, precision="mixed").cpu().numpy()
    assert np.max(np.abs(SAm - ref)) <= 64 * 2.0 ** -23 * np.abs(A).sum(axis=0).max()


@pytest.mark.parametrize("n,d,m", [(4096, 256, 256), (1000, 37, 50), (300, 5, 300)])
def test_gaussian_plain(n, d, m):
    mihs = _mihs()
    A = _rand(n, d, 4)
    ref = sketches.gaussian_sketch(A, m, 7)
    announce(f"gaussian plain n={n} d={d} m={m}")
    SA = mihs.mihs_sketch(to_dev(A), "gaussian", m, 7).cpu().numpy()
    scale = np.sqrt(n / m) * np.abs(A).max()
    assert np.max(np.abs(SA - ref)) <= 1e-12 * scale


@pytest.mark.parametrize("n,d,m", [(4096, 256, 256), (1000, 37, 50), (2048, 130, 384)])
def test_gaussian_mixed_bf16(n, d, m):
    """BF16 S and BF16 A on the matrix cores, FP32 accumulation: compare with
    the BF16-rounded product, within FP32 accumulation error."""
    mihs = _mihs()
    A = _rand(n, d, 4)
    ref = sketches.gaussian_sketch_bf16(A, m, 7)
    announce(f"gaussian mixed n={n} d={d} m={m}")
    SA = mihs.mihs_sketch(to_dev(A), "gaussian", m, 7, precision="mixed")
    assert SA.dtype == torch.float32
    SA = SA.cpu().numpy().astype(np.float64)
    S = np.abs(sketches.gaussian_matrix(m, n, 7))
    bound = (n + 2) * 2.0 ** -24 * (S @ np.abs(A)) + 1e-30
    assert np.all(np.abs(SA - ref) <= bound)
    # and it is a BF16-accurate sketch of the exact product
    exact = sketches.gaussian_sketch(A, m, 7)
    assert rel(SA, exact) < 2e-2


def test_gaussian_mixed_entries_within_one_bf16_unit():
    """The mixed path draws its Gaussian entries in FP32 (hardware log2 / sine /
    cosine) and rounds them to BF16: sketching the identity exposes S itself,
    which must equal the oracle's FP64 draws rounded to BF16 except for rare
    entries where the FP32 draw's error crosses a rounding boundary: one BF16
    unit, or, near the zeros of sine and cosine, the draw's absolute error
    (the hardware sine and cosine are accurate to a few units of 2^-22 in
    absolute terms; with rad <= 7 that is below 2^-16, i.e. below 2^-16 of an
    entry's typical size 1/sqrt(m))."""
    mihs = _mihs()
    n, m, seed = 1024, 256, 21
    A = np.eye(n)
    announce("gaussian mixed entries (identity)")
    S_gpu = mihs.mihs_sketch(to_dev(A), "gaussian", m, seed, precision="mixed")
    S_gpu = S_gpu.cpu().numpy().astype(np.float64)
    idx = np.arange(m * n, dtype=np.int64).reshape(m, n)
    S_ref = sketches.bf16_round(sketches.gaussian_entries(seed, 0, idx) / math.sqrt(m))
    ulp = np.exp2(np.floor(np.log2(np.maximum(np.abs(S_ref), 1e-30))) - 7)
    diff = np.abs(S_gpu - S_ref)
    bound = np.maximum(ulp * 1.0000001, 2.0 ** -16 / math.sqrt(m))
    assert np.all(diff <= bound), float((diff / bound).max())
    assert np.count_nonzero(diff) <= 1e-3 * m * n, np.count_nonzero(diff)


def test_count_gauss_plain_and_mixed():
    mihs = _mihs()
    n, d, m1, m2 = 30000, 48, 512, 128
    A = _rand(n, d, 6, np.float32)
    ref = sketches.count_gauss_sketch(A, m1, m2, 99)
    announce("count_gauss plain")
    SA = mihs.mihs_sketch(to_dev(A), "count_gauss", m1, 99, m2=m2).cpu().numpy()
    assert SA.shape == (m2, d)
    assert rel(SA, ref) <= 1e-13
    announce("count_gauss mixed")
    SAm = mihs.mihs_sketch(to_dev(A), "count_gauss", m1, 99, m2=m2, precision="mixed")
    SAm = SAm.cpu().numpy().astype(np.float64)
    CA = sketches.countsketch(A, m1, 99)
    # mixed second stage: BF16 Gaussian entries times the FP32 bucket sums kept
    # to FP32 accuracy (three BF16 terms), i.e. bf16(G) CA -- not bf16(G) bf16(CA)
    idx = np.arange(m2 * m1, dtype=np.int64).reshape(m2, m1)
    G16 = sketches.bf16_round(sketches.gaussian_entries(99, 1, idx) / math.sqrt(m2))
    ref_split = G16 @ CA
    ref_rounded = sketches.gaussian_sketch_bf16(CA, m2, 99, stream=1)
    assert rel(SAm, ref_split) <= 2e-4
    assert rel(ref_rounded, ref_split) > 5e-4  # the bound above tells the two apart
    assert rel(SAm, ref) <= 2e-2
