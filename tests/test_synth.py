"""Pins for the seeded input generator: code construction, encoding, RNG, channel."""
import itertools
import math
from collections import Counter

import numpy as np
import pytest

import synth

EBCH = [(8, 4), (16, 11), (32, 26), (64, 57), (128, 120)]


def _weight4_count(code):
    # 4-subsets of columns whose syndromes XOR to zero, counted through pairs with equal XOR:
    # each such 4-set splits into 3 pairs-of-pairs; pairs sharing a bit would need equal columns.
    cols = code.hcols
    cnt = Counter()
    for i in range(code.n):
        for j in range(i + 1, code.n):
            cnt[cols[i] ^ cols[j]] += 1
    tot = sum(c * (c - 1) // 2 for c in cnt.values())
    assert tot % 3 == 0
    return tot // 3


@pytest.mark.parametrize("n,k", EBCH)
def test_extended_hamming_weight_structure(n, k):
    code = synth.ebch(n, k)
    assert code.r == n - k and code.is_even
    cols = code.hcols
    assert all(c != 0 for c in cols) and len(set(cols)) == n      # no weight 1 or 2 codewords
    assert all(bin(c >> (n - k - 1)).count("1") == 1 for c in cols)  # all-ones row => no odd weight
    # extended Hamming codes: A_4 = n(n-1)(n-2)/24
    assert _weight4_count(code) == n * (n - 1) * (n - 2) // 24


def test_ebch_16_7_min_distance_6():
    code = synth.ebch(16, 7)
    G = code.G.astype(int)
    ws = [int(((np.array(m) @ G) % 2).sum()) for m in itertools.product([0, 1], repeat=code.k)]
    assert min(w for w in ws if w) == 6 and all(w % 2 == 0 for w in ws)


@pytest.mark.parametrize("n,k", EBCH)
def test_encoders_satisfy_parity_checks(n, k):
    code = synth.ebch(n, k)
    H = code.H().astype(np.int64)
    u = synth.info_bits(3, np.arange(50), k)
    c = synth.encode(code, u)
    assert not np.any((c.astype(np.int64) @ H.T) % 2)
    assert np.array_equal(c[:, list(code.info_pos)], u)
    if n <= 64:
        U = synth.info_bits(4, np.arange(5), k * k).reshape(-1, k, k)
        C = synth.encode_product(code, U).astype(np.int64)
        assert not np.any((C @ H.T) % 2)                       # rows
        assert not np.any((np.swapaxes(C, 1, 2) @ H.T) % 2)    # columns
        ip = list(code.info_pos)
        assert np.array_equal(C[:, ip][:, :, ip], U)


def test_generic_generator_code_matches_membership():
    base = synth.ebch(16, 11)
    code = synth.code_from_generator("copy", base.G, base.info_pos)
    H = code.H().astype(np.int64)
    cw = synth.encode(base, synth.info_bits(0, np.arange(20), 11)).astype(np.int64)
    assert not np.any((cw @ H.T) % 2)
    assert code.is_even


def test_splitmix_reference_values():
    # SplitMix64 seeded with 0: first outputs of the public-domain reference generator
    # (state += 0x9E3779B97F4A7C15; mix), computed here with Python integers.
    state = 0
    ref = []
    for _ in range(3):
        state = (state + 0x9E3779B97F4A7C15) & synth.MASK64
        ref.append(synth._mix_int(state))
    assert ref[0] == 0xE220A8397B1DCDAF
    assert ref[1] == 0x6E789E6AA1B965F4
    assert ref[2] == 0x06C45D188009454F


def test_streams_are_counter_based_and_deterministic():
    a = synth.gaussians(7, np.arange(10), 33)
    b = synth.gaussians(7, np.array([3, 8]), 33)
    assert np.array_equal(a[[3, 8]], b)
    assert not np.array_equal(a[0], a[1])
    assert np.array_equal(synth.info_bits(1, [5], 40), synth.info_bits(1, [5], 40))


def test_gaussian_moments():
    z = synth.gaussians(11, np.arange(200), 5000).ravel()
    assert abs(z.mean()) < 0.005 and abs(z.var() - 1.0) < 0.01
    assert abs(np.mean(z ** 4) - 3.0) < 0.05


def test_channel_llr_scale():
    code = synth.ebch(32, 26)
    llr, cw, _ = synth.product_frames(code, 3.0, 0, np.arange(200))
    R = 26 * 26 / (32 * 32)
    s2 = synth.sigma2(3.0, R)
    assert math.isclose(s2, 1 / (2 * R * 10 ** 0.3))
    x = 1 - 2 * cw.astype(float)
    r = llr * s2 / 2
    noise = (r - x).ravel()
    assert abs(noise.var() / s2 - 1) < 0.01
    # raw hard-decision bit error rate equals Q(1/sigma)
    ber = np.mean((llr < 0) != (cw == 1))
    q = 0.5 * math.erfc(1 / math.sqrt(2 * s2))
    assert abs(ber - q) < 0.003


# ---------------------------------------------------------------- block Rician fading with QPSK
def test_rician_noiseless_signs_follow_the_codeword():
    code = synth.ebch(32, 26)
    llr, cw, _ = synth.rician_product_frames(code, 80.0, 8.0, 256, 3, np.arange(6))
    assert np.all((llr < 0) == (cw == 1))


@pytest.mark.parametrize("K", [0.0, 6.0])
def test_rician_llr_statistics(K):
    """All-zero codewords: every LLR has mean 2 E|H|^2 / sigma^2 = 2 / sigma^2 (E|H|^2 = 1 for any
    K), and the per-coherence-block mean LLR spreads like |H|^2, whose variance is
    (2K + 1) / (K + 1)^2 for a Rician factor K (1 for Rayleigh)."""
    F, N, nc, rate, eb = 4000, 1024, 64, 0.5, 4.0
    s2 = 1.0 / (2.0 * rate * 10.0 ** (eb / 10.0))
    ids = np.arange(F, dtype=np.uint64)
    llr = synth.rician_qpsk_llr(np.zeros((F, N), np.uint8), eb, rate, K, nc, 9, ids)
    mu = 2.0 / s2
    assert abs(llr.mean() / mu - 1.0) < 0.02
    # regroup code bits by coherence block: interleaved bit i is code bit perm[i], symbol i // 2
    perm = np.argsort(synth.splitmix_stream(9, ids, 3, N), axis=1, kind="stable")
    inter = np.take_along_axis(llr, perm, axis=1)
    block_mean = inter.reshape(F, N // (2 * nc), 2 * nc).mean(axis=2) / mu
    expect = (2 * K + 1) / (K + 1) ** 2 + s2 / (2 * nc)      # |H|^2 spread plus the noise left in the mean
    assert abs(block_mean.var() / expect - 1.0) < 0.08


def test_rician_large_k_is_awgn():
    """K -> infinity leaves H = 1: each LLR is 2 (x + n) / sigma^2 with n ~ N(0, sigma^2), as for BPSK."""
    F, N, rate, eb = 2000, 1024, 0.5, 3.0
    s2 = 1.0 / (2.0 * rate * 10.0 ** (eb / 10.0))
    llr = synth.rician_qpsk_llr(np.zeros((F, N), np.uint8), eb, rate, 1e12, 256, 4, np.arange(F))
    assert abs(llr.mean() / (2.0 / s2) - 1.0) < 0.01
    assert abs(llr.var() / (4.0 / s2) - 1.0) < 0.02
