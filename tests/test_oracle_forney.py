"""Pins of Forney's list-based soft output (eq. missingterm), the comparator of the paper's Fig. 2.

What fixes it, independently of its own arithmetic:
* with the whole codebook in the list, the approximation is no approximation: it equals the exact
  posterior of formula (forney), here summed by brute force over every codeword from the Gaussian
  channel densities of the received signal;
* its estimate for the most likely list entry is never below 1/L (stated next to eq. missingterm);
* at 2 dB with a list of 5 predicting the error of the first 4, the empirical list-BLER lies far
  above the prediction, on the paper's dashed Fig. 2 curves, while SOGRAND's prediction for the
  same words stays on the diagonal (its own calibration test).
"""
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig2_forney_list_bler.txt")


def paper_points():
    pts = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        nk, p, e = line.split()
        pts.setdefault(tuple(int(x) for x in nk.split(",")), []).append((float(p), float(e)))
    return pts


def in_first(llr, cw, found_z, n_found, lprime):
    """Whether the transmitted codeword is among the first lprime list entries."""
    y = (llr < 0).astype(np.uint8)
    hit = np.zeros(len(cw), dtype=bool)
    for l in range(lprime):
        hit |= (l < n_found) & np.all((y ^ found_z[:, l]) == cw, axis=1)
    return hit


def binned(pred, hit):
    """(mean prediction, empirical miss rate, misses, words) per half-decade bin of the prediction."""
    ok = np.isfinite(pred) & (pred > 0)
    bins = np.floor(-2 * np.log10(np.where(ok, pred, 1.0))).astype(int)
    rows = []
    for b in range(0, 12):
        sel = ok & (bins == b)
        if sel.sum() == 0:
            continue
        errs = int((~hit[sel]).sum())
        rows.append((float(pred[sel].mean()), errs / int(sel.sum()), errs, int(sel.sum())))
    return rows


def curve_at(rows, x, min_errs=40):
    """The empirical curve at prediction x, interpolated on log-log axes between the two bins around
    it (both with at least min_errs misses); None outside the measured range."""
    pts = sorted((p, e) for p, e, errs, _ in rows if errs >= min_errs)
    for (p0, e0), (p1, e1) in zip(pts, pts[1:]):
        if p0 <= x <= p1:
            t = np.log(x / p0) / np.log(p1 / p0)
            return float(np.exp(np.log(e0) + t * np.log(e1 / e0)))
    return None


def check_forney_curve(nk, rows, factor):
    """Shared by the oracle and GPU calibration tests: the curve lies far above the diagonal and on
    the paper's points within `factor`.  Returns the number of paper points compared."""
    for pred, emp, errs, cnt in rows:
        if errs >= 40 and pred < 0.1:
            assert emp >= 2.0 * pred, (nk, pred, emp, errs, cnt)
    checked = 0
    for px, py in paper_points()[nk]:
        got = curve_at(rows, px)
        if got is None:
            continue
        checked += 1
        assert py / factor <= got <= py * factor, (nk, px, py, got)
    return checked


def test_full_codebook_list_is_the_exact_posterior():
    code = synth.ebch(8, 4)
    words = 40
    ebn0 = 1.0
    llr, cw, _ = synth.component_words(code, ebn0, 17, np.arange(words))
    # all 16 codewords: every codeword lies in the parity class that is searched, 128 patterns
    out = oracle.decode_component(code, llr, 16, 128, want_z=True)
    assert np.all(out["n_found"] == 16)
    p = oracle.forney_app(llr, out["found_z"], out["n_found"])
    # brute force: every length-8 word with zero syndrome, Gaussian densities of r = x + noise
    H = code.H().astype(np.int64)
    allw = ((np.arange(256)[:, None] >> np.arange(8)[None, :]) & 1).astype(np.int64)
    book = allw[~np.any((allw @ H.T) % 2, axis=1)]
    assert len(book) == 16
    s2 = 1.0 / (2.0 * (4 / 8) * 10.0 ** (ebn0 / 10.0))
    r = llr * s2 / 2.0
    y = (llr < 0).astype(np.int64)
    for w in range(words):
        dens = np.array([np.exp(-np.sum((r[w] - (1.0 - 2.0 * c)) ** 2) / (2.0 * s2)) for c in book])
        post = dens / dens.sum()
        for l in range(16):
            c = y[w] ^ out["found_z"][w, l]
            j = int(np.flatnonzero(np.all(book == c, axis=1))[0])
            assert abs(p[w, l] - post[j]) <= 1e-12 * max(post[j], 1e-300) + 1e-15, (w, l)
    # and the transmitted codeword's posterior is what is left out of a shorter list
    assert np.all(oracle.forney_list_bler(llr, out["found_z"], out["n_found"], 16) < 1e-12)


def test_most_likely_entry_at_least_one_over_list_size():
    code = synth.ebch(32, 26)
    llr, _, _ = synth.component_words(code, 2.0, 18, np.arange(3000))
    for L in (2, 5):
        out = oracle.decode_component(code, llr, L, 10 ** 5, want_z=True)
        p = oracle.forney_app(llr, out["found_z"], out["n_found"])
        full = out["n_found"] == L
        assert full.sum() > 2900
        np.testing.assert_allclose(p[full].sum(axis=1), 1.0, rtol=0, atol=1e-14)
        assert np.all(p[full].max(axis=1) >= 1.0 / L - 1e-15)
        # ... and the prediction for the first L - 1 is the last entry's share
        pl = oracle.forney_list_bler(llr, out["found_z"], out["n_found"], L - 1)
        np.testing.assert_allclose(pl[full], p[full, L - 1], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("nk,words", [((16, 11), 60000), ((32, 26), 60000), ((64, 57), 40000)])
def test_forney_list_bler_matches_fig2(nk, words):
    code = synth.ebch(*nk)
    llr, cw, _ = synth.component_words(code, 2.0, 101, np.arange(words))
    out = oracle.decode_component(code, llr, 5, 10 ** 5, want_z=True)
    pred = oracle.forney_list_bler(llr, out["found_z"], out["n_found"], 4)
    rows = binned(pred, in_first(llr, cw, out["found_z"], out["n_found"], 4))
    # The tolerance is wider than for SOGRAND's own curve: a list-based estimate also carries the
    # list decoder's misses, and the paper's lists come from a more accurate query order.
    assert check_forney_curve(nk, rows, factor=1.6) >= 3
