"""Pins for the oracle's SOGRAND component and product decoding.

Each check compares the oracle with something it does not compute itself:
brute force over every pattern / codeword of tiny codes, Gaussian channel
likelihoods evaluated from the received samples, closed forms, and exact
symmetries of the method.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth


def hamming15():
    base = synth.ebch(16, 11)
    G = base.G[:, :15]
    return synth.code_from_generator("Hamming[15,11]", G, base.info_pos)


def words(code, ebn0, seed, count):
    llr, cw, _ = synth.component_words(code, ebn0, seed, np.arange(count))
    s2 = synth.sigma2(ebn0, code.k / code.n)
    r = llr * s2 / 2.0
    return llr, cw, r, s2


def codebook(code):
    msgs = np.array(list(itertools.product([0, 1], repeat=code.k)), dtype=np.int64)
    return ((msgs @ code.G.astype(np.int64)) & 1).astype(np.uint8)


def flip_probs(r, s2):
    """P(hard decision of bit i is wrong | r_i) from the Gaussian densities."""
    xhat = np.where(r < 0, -1.0, 1.0)
    f_same = np.exp(-(r - xhat) ** 2 / (2 * s2))
    f_other = np.exp(-(r + xhat) ** 2 / (2 * s2))
    return f_other / (f_same + f_other)


class Brute:
    """Every pattern of the eligible class with its query number and exact probability."""

    def __init__(self, code, llr, r, s2):
        n = code.n
        self.y = (llr < 0).astype(np.uint8)
        a = np.abs(llr)
        order = sorted(range(n), key=lambda i: (a[i], i))
        rank = np.empty(n, dtype=np.int64)
        rank[order] = np.arange(1, n + 1)
        par = int(self.y.sum() % 2)
        pf = flip_probs(r, s2)
        masks = np.arange(1 << n, dtype=np.int64)
        bits = ((masks[:, None] >> np.arange(n)) & 1).astype(np.uint8)
        w = bits.sum(1)
        if code.is_even:
            keep = (w % 2) == par
            bits, w, masks = bits[keep], w[keep], masks[keep]
        W = bits.astype(np.int64) @ rank
        tuples = [tuple(sorted(rank[b.astype(bool)])) for b in bits]
        idx = sorted(range(len(masks)), key=lambda t: (W[t], w[t], tuples[t]))
        self.q_of_mask = {int(masks[t]): qn + 1 for qn, t in enumerate(idx)}
        logp = np.where(bits == 1, np.log(pf), np.log1p(-pf)).sum(1)
        self.p_of_mask = {int(m): float(np.exp(lp)) for m, lp in zip(masks, logp)}
        self.count = len(masks)
        self.par = par
        self.pf = pf

    def mask_of(self, z):
        return int(sum(int(b) << i for i, b in enumerate(z)))

    def expected_list(self, code, L, qcap):
        cb = codebook(code)
        hits = []
        for c in cb:
            m = self.mask_of(self.y ^ c)
            q = self.q_of_mask[m]
            if q <= qcap:
                hits.append((q, m))
        hits.sort()
        return hits[:L]


CASES = [((8, 4), 1.0, 0), ((8, 4), 4.0, 1), ((16, 11), 2.0, 2), ((16, 11), 5.0, 3)]


@pytest.mark.parametrize("nk,ebn0,seed", CASES)
@pytest.mark.parametrize("L,qcap", [(1, 10 ** 6), (4, 10 ** 6), (4, 30), (3, 7)])
def test_list_and_query_numbers_match_bruteforce(nk, ebn0, seed, L, qcap):
    code = synth.ebch(*nk)
    llr, _, r, s2 = words(code, ebn0, seed, 6)
    out = oracle.decode_component(code, llr, L, qcap, want_z=True, want_diag=True)
    for wd in range(llr.shape[0]):
        B = Brute(code, llr[wd], r[wd], s2)
        exp = B.expected_list(code, L, qcap)
        nf = int(out["n_found"][wd])
        assert nf == len(exp)
        assert list(out["found_q"][wd, :nf]) == [q for q, _ in exp]
        for l in range(nf):
            assert B.mask_of(out["found_z"][wd, l]) == exp[l][1]
        # queries tested: the L-th hit, else the cap, else the whole class
        Q = exp[-1][0] if nf == L else min(qcap, B.count)
        assert int(out["n_queries"][wd]) == Q
        # queried, not-found and parity-class masses against the brute-force sums
        S = sum(p for m, p in B.p_of_mask.items() if B.q_of_mask[m] <= Q)
        M = sum(p for m, p in B.p_of_mask.items() if B.q_of_mask[m] > Q)
        Ppar = sum(B.p_of_mask.values())
        p0, Sd, Md, Pd, exhausted = out["diag"][wd]
        assert exhausted == (1.0 if Q == B.count else 0.0)
        assert math.isclose(Sd, S, rel_tol=1e-12)
        assert math.isclose(Pd, Ppar, rel_tol=1e-12)
        assert math.isclose(Md, M, rel_tol=1e-10, abs_tol=1e-300)
        assert math.isclose(p0, float(np.prod(1 - B.pf)), rel_tol=1e-12)
        # closed form of the parity-class mass: (1 + (-1)^rho prod (1 - 2 p_i)) / 2
        closed = 0.5 * (1 + (-1) ** B.par * np.prod(1 - 2 * B.pf))
        assert math.isclose(Pd, closed, rel_tol=1e-12)


def test_non_even_code_queries_all_weights_and_uses_full_mass():
    code = hamming15()
    assert not code.is_even and not oracle.code_is_even(code)
    llr, _, r, s2 = words(code, 3.0, 5, 5)
    out = oracle.decode_component(code, llr, 3, 200, want_z=True, want_diag=True)
    for wd in range(5):
        B = Brute(code, llr[wd], r[wd], s2)
        exp = B.expected_list(code, 3, 200)
        nf = int(out["n_found"][wd])
        assert list(out["found_q"][wd, :nf]) == [q for q, _ in exp]
        Q = int(out["n_queries"][wd])
        M = sum(p for m, p in B.p_of_mask.items() if B.q_of_mask[m] > Q)
        assert math.isclose(out["diag"][wd, 2], M, rel_tol=1e-10)
        assert math.isclose(out["diag"][wd, 3], 1.0, rel_tol=1e-15)
        # P_nf from Corollary 1 with phi = (2^k - 1)/(2^n - 1)
        phi = (2 ** code.k - 1) / (2 ** code.n - 1)
        pz = [B.p_of_mask[B.mask_of(z)] for z in out["found_z"][wd, :nf]]
        D = sum(pz) + M * phi
        assert math.isclose(out["p_notfound"][wd], M * phi / D, rel_tol=1e-10)
        for l in range(nf):
            assert math.isclose(out["p_found"][wd, l], pz[l] / D, rel_tol=1e-10)


@pytest.mark.parametrize("nk,ebn0", [((8, 4), 0.0), ((8, 4), 3.0), ((16, 11), 1.0), ((16, 11), 4.0)])
def test_exhaustive_list_gives_exact_bitwise_app(nk, ebn0):
    """A list longer than the codebook makes the search run through the whole parity class:
    every codeword is found, the not-found mass is zero, Corollary 1 reduces to the exact
    codeword posterior and eq. (LLRi) to the exact bitwise APP LLR (Forney's formula)."""
    code = synth.ebch(*nk)
    llr, _, r, s2 = words(code, ebn0, 9, 4)
    L = 1 << code.k
    out = oracle.decode_component(code, llr, L + 1, 1 << (code.n - 1), want_diag=True)
    cb = codebook(code).astype(np.float64)
    x = 1.0 - 2.0 * cb
    for wd in range(4):
        assert out["n_found"][wd] == L and out["n_queries"][wd] == 1 << (code.n - 1)
        # every pattern of the class was tested: the untested mass is exactly zero
        assert out["diag"][wd, 2] == 0.0 and out["diag"][wd, 4] == 1.0
        logf = -((r[wd][None, :] - x) ** 2).sum(1) / (2 * s2)
        logf -= logf.max()
        f = np.exp(logf)
        num = (f[:, None] * (cb == 0)).sum(0)
        den = (f[:, None] * (cb == 1)).sum(0)
        exact = np.log(num) - np.log(den)
        err = np.abs(out["llr_app"][wd] - exact) / np.maximum(1.0, np.abs(exact))
        assert err.max() <= 1e-12
        assert out["p_notfound"][wd] == 0.0


@pytest.mark.parametrize("nk,ebn0", [((16, 11), 2.0), ((32, 26), 3.0), ((64, 57), 3.0)])
def test_soft_output_invariants(nk, ebn0):
    code = synth.ebch(*nk)
    llr, _, _, _ = words(code, ebn0, 13, 40)
    for L, qcap in [(1, 1000), (4, 1000), (4, 20)]:
        out = oracle.decode_component(code, llr, L, qcap)
        tot = out["p_found"].sum(1) + out["p_notfound"]
        np.testing.assert_allclose(tot, 1.0, rtol=1e-13)
        assert np.all(out["p_found"] >= 0) and np.all(out["p_notfound"] >= 0)
        np.testing.assert_array_equal(out["hard"], (out["llr_app"] < 0).astype(np.uint8))
        np.testing.assert_allclose(out["llr_ext"], out["llr_app"] - llr, rtol=0, atol=1e-12)
        # P_i are ratios of p(z_i|r): the first found (most likely queried) is the largest
        assert np.all(out["n_queries"] <= qcap)


def test_empty_list_returns_soft_input():
    code = synth.ebch(64, 57)
    llr, _, _, _ = words(code, 1.0, 17, 200)
    out = oracle.decode_component(code, llr, 4, 1)
    empty = out["n_found"] == 0
    assert empty.sum() > 50
    assert np.all(out["p_notfound"][empty] == 1.0)
    np.testing.assert_allclose(out["llr_app"][empty], llr[empty], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(out["llr_ext"][empty], 0.0, atol=1e-12)


@pytest.mark.parametrize("nk", [(16, 11), (32, 26), (64, 57), (128, 120)])
def test_codeword_translation_equivariance(nk):
    """Flipping the LLR signs on the support of a codeword translates the whole search:
    same ranks, syndromes and parity, so the same query numbers, and the APP LLRs flip sign."""
    code = synth.ebch(*nk)
    llr, _, _, _ = words(code, 3.0, 21, 12)
    c = synth.encode(code, synth.info_bits(99, np.arange(12), code.k))
    llr2 = np.where(c == 1, -llr, llr)
    a = oracle.decode_component(code, llr, 4, 3000, want_z=True)
    b = oracle.decode_component(code, llr2, 4, 3000, want_z=True)
    for key in ("n_queries", "n_found", "found_q", "found_z", "p_found", "p_notfound"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(b["llr_app"], np.where(c == 1, -a["llr_app"], a["llr_app"]))


def test_bit_permutation_equivariance():
    code = synth.ebch(32, 26)
    llr, _, _, _ = words(code, 2.5, 23, 10)
    perm = np.random.default_rng(0).permutation(code.n)
    pcode = synth.code_from_generator("perm", code.G[:, perm], [int(np.where(perm == p)[0][0]) for p in code.info_pos])
    a = oracle.decode_component(code, llr, 4, 2000)
    b = oracle.decode_component(pcode, llr[:, perm], 4, 2000)
    np.testing.assert_array_equal(a["found_q"], b["found_q"])
    np.testing.assert_array_equal(a["n_queries"], b["n_queries"])
    np.testing.assert_allclose(b["llr_app"], a["llr_app"][:, perm], rtol=1e-12, atol=1e-12)


def test_ties_are_broken_by_lower_index():
    code = synth.ebch(8, 4)
    llr = np.array([[1.0, -1.0, 1.0, 2.0, -2.0, 3.0, 3.0, 0.5]])
    out = oracle.decode_component(code, llr, 4, 128, want_z=True)
    B = Brute(code, llr[0], llr[0] / 2, 1.0)   # ranks from |llr| with index tie-break
    exp = B.expected_list(code, 4, 128)
    assert list(out["found_q"][0, :out["n_found"][0]]) == [q for q, _ in exp]


def test_product_noiseless_frame_stops_after_first_row_pass():
    code = synth.ebch(32, 26)
    U = synth.info_bits(5, np.arange(3), code.k ** 2).reshape(3, code.k, code.k)
    C = synth.encode_product(code, U)
    llr = 8.0 * (1.0 - 2.0 * C.astype(np.float64))
    out = oracle.decode_product(code, llr, 4, 1000, 4)
    assert np.all(out["success"] == 1) and np.all(out["half_iters"] == 1)
    np.testing.assert_array_equal(out["hard"], C)


def test_product_translation_equivariance_and_threads():
    code = synth.ebch(32, 26)
    llr, cw, _ = synth.product_frames(code, 2.75, 31, np.arange(16))
    U = synth.info_bits(6, np.arange(16), code.k ** 2).reshape(16, code.k, code.k)
    C = synth.encode_product(code, U)
    a = oracle.decode_product(code, llr, 4, 1000, 4, want_app=True)
    b = oracle.decode_product(code, np.where(C == 1, -llr, llr), 4, 1000, 4, want_app=True, nthreads=4)
    for key in ("success", "half_iters", "sum_queries", "sum_max_queries"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(b["hard"], a["hard"] ^ C)
    np.testing.assert_array_equal(b["llr_app"], np.where(C == 1, -a["llr_app"], a["llr_app"]))


def test_product_success_means_valid_product_codeword():
    code = synth.ebch(32, 26)
    llr, cw, _ = synth.product_frames(code, 2.5, 0, np.arange(30))
    out = oracle.decode_product(code, llr, 4, 1000, 4)
    H = code.H().astype(np.int64)
    for f in range(30):
        Cf = out["hard"][f].astype(np.int64)
        valid = not np.any((Cf @ H.T) % 2) and not np.any((Cf.T @ H.T) % 2)
        assert valid == bool(out["success"][f])
    assert out["success"].mean() > 0.5
    assert np.all((out["half_iters"] >= 1) & (out["half_iters"] <= 8))
    fails = out["success"] == 0
    assert np.all(out["half_iters"][fails] == 8)


def test_product_store_f32_rounds_exchange():
    code = synth.ebch(32, 26)
    llr, _, _ = synth.product_frames(code, 3.0, 1, np.arange(8))
    llr32 = llr.astype(np.float32).astype(np.float64)
    a = oracle.decode_product(code, llr32, 4, 1000, 4, store_f32=True)
    b = oracle.decode_product(code, llr32, 4, 1000, 4, store_f32=False)
    # rounding the exchanged LLRs to binary32 perturbs them only slightly
    assert np.mean(a["hard"] == b["hard"]) > 0.999
