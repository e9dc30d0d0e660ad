"""Pins for the list-BLER stop of the oracle: the search ends after the first codeword whose
list, with the mass tested up to its query, has a predicted list-BLER (Corollary 1) below
the threshold.  Checked against brute-force masses of tiny codes, the limiting thresholds
and the prefix structure of the lists."""
import math

import numpy as np
import pytest

import oracle
import synth
from test_oracle_decode import Brute, codebook, words


def expected_stop(code, B, L, qcap, tau):
    """List size and query count from brute-force masses: stop at the first hit i < L whose
    not-found probability M_i phi / (sum_{l<=i} p_l + M_i phi) is below tau."""
    hits = B.expected_list(code, L, qcap)
    n, k = code.n, code.k
    phi = (2.0 ** k - 1) / ((2.0 ** (n - 1) if code.is_even else 2.0 ** n) - 1)
    for i, (q, _) in enumerate(hits, start=1):
        if i == L:
            break
        M = sum(p for m, p in B.p_of_mask.items() if B.q_of_mask[m] > q)
        P = sum(B.p_of_mask[m] for _, m in hits[:i])
        pnf = M * phi / (P + M * phi)
        if math.isclose(pnf, tau, rel_tol=1e-8):
            return None   # too close to the threshold to pin
        if pnf < tau:
            return i, q
    if len(hits) == L:
        return L, hits[-1][0]
    return len(hits), min(qcap, B.count)


CASES = [((8, 4), 1.0, 0), ((8, 4), 3.0, 1), ((16, 11), 2.0, 2), ((16, 11), 4.0, 3)]


@pytest.mark.parametrize("nk,ebn0,seed", CASES)
@pytest.mark.parametrize("tau", [0.3, 1e-2, 1e-4])
def test_stop_point_matches_bruteforce(nk, ebn0, seed, tau):
    code = synth.ebch(*nk)
    llr, _, r, s2 = words(code, ebn0, seed, 8)
    L, qcap = 4, 10 ** 6
    out = oracle.decode_component(code, llr, L, qcap, want_z=True, pstop=tau)
    checked = 0
    for wd in range(llr.shape[0]):
        B = Brute(code, llr[wd], r[wd], s2)
        exp = expected_stop(code, B, L, qcap, tau)
        if exp is None:
            continue
        nf, Q = exp
        assert int(out["n_found"][wd]) == nf, wd
        assert int(out["n_queries"][wd]) == Q, wd
        hits = B.expected_list(code, L, qcap)
        assert list(out["found_q"][wd, :nf]) == [q for q, _ in hits[:nf]]
        checked += 1
    assert checked >= 6


def test_zero_threshold_is_no_stop_and_one_is_a_single_codeword():
    code = synth.ebch(32, 26)
    llr, _, _, _ = words(code, 3.0, 11, 200)
    base = oracle.decode_component(code, llr, 4, 1000)
    off = oracle.decode_component(code, llr, 4, 1000, pstop=0.0)
    for key in base:
        if base[key] is not None:
            np.testing.assert_array_equal(base[key], off[key], err_msg=key)
    one = oracle.decode_component(code, llr, 4, 1000, pstop=1.0)
    l1 = oracle.decode_component(code, llr, 1, 1000)
    np.testing.assert_array_equal(one["n_found"], l1["n_found"])
    np.testing.assert_array_equal(one["n_queries"], l1["n_queries"])
    np.testing.assert_array_equal(one["found_q"][:, :1], l1["found_q"])
    np.testing.assert_array_equal(one["llr_app"], l1["llr_app"])


def test_lists_shrink_as_the_threshold_grows_and_stay_prefixes():
    code = synth.ebch(32, 26)
    llr, _, _, _ = words(code, 2.5, 12, 300)
    prev = oracle.decode_component(code, llr, 4, 1000, pstop=0.0)
    assert np.all(prev["n_found"] >= 1)
    for tau in (1e-6, 1e-4, 1e-2, 0.5):
        cur = oracle.decode_component(code, llr, 4, 1000, pstop=tau)
        assert np.all(cur["n_found"] <= prev["n_found"])
        assert np.all(cur["n_queries"] <= prev["n_queries"])
        for wd in range(llr.shape[0]):
            nf = int(cur["n_found"][wd])
            assert list(cur["found_q"][wd, :nf]) == list(prev["found_q"][wd, :nf])
        # a stopped list's predicted list-BLER is below the threshold
        stopped = cur["n_found"] < prev["n_found"]
        assert np.all(cur["p_notfound"][stopped] < tau * (1 + 1e-9))
        prev = cur


def test_product_with_threshold_one_equals_single_codeword_lists():
    code = synth.ebch(16, 11)
    llr, _, _ = synth.product_frames(code, 2.5, 13, np.arange(20))
    a = oracle.decode_product(code, llr, 4, 1000, 4, pstop=1.0)
    b = oracle.decode_product(code, llr, 1, 1000, 4)
    for key in ("hard", "success", "half_iters", "sum_queries", "sum_max_queries"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)


def test_threshold_outside_unit_interval_is_rejected():
    code = synth.ebch(16, 11)
    llr, _, _, _ = words(code, 3.0, 1, 2)
    with pytest.raises(ValueError):
        oracle.decode_component(code, llr, 4, 100, pstop=-0.1)
    with pytest.raises(ValueError):
        oracle.decode_component(code, llr, 4, 100, pstop=1.5)
