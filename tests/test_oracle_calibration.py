"""Statistical pins of the oracle's soft output against the paper's Figs. 2 and 4.

The paper shows that the predicted probability that the transmitted codeword is
not in the list (eq. app_approxlist) matches the empirical list-BLER for eBCH
codes (L = 4, 2 dB).  The oracle's prediction, binned per half decade, must be
as well calibrated as the paper's own points: a wrong hit probability phi, a
dropped mass term or a wrong parity-class reading shifts the curve off the
diagonal by a large factor.
"""
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig2_list_bler_calibration.txt")
GOLDEN4 = os.path.join(os.path.dirname(__file__), "golden", "fig4_bitwise_so_calibration.txt")


def paper_points():
    pts = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        nk, p, e = line.split()
        pts.setdefault(tuple(int(x) for x in nk.split(",")), []).append((float(p), float(e)))
    return pts


def calibration(code, words, seed):
    llr, cw, _ = synth.component_words(code, 2.0, seed, np.arange(words))
    out = oracle.decode_component(code, llr, 4, 10 ** 5, want_z=True)
    y = (llr < 0).astype(np.uint8)
    in_list = np.zeros(words, dtype=bool)
    for l in range(4):
        ok = l < out["n_found"]
        match = np.all((y ^ out["found_z"][:, l]) == cw, axis=1)
        in_list |= ok & match
    pred = out["p_notfound"]
    bins = np.floor(-2 * np.log10(np.maximum(pred, 1e-300))).astype(int)
    rows = []
    for b in range(0, 8):
        sel = bins == b
        if sel.sum() == 0:
            continue
        errs = int((~in_list[sel]).sum())
        rows.append((float(pred[sel].mean()), errs / sel.sum(), errs, int(sel.sum())))
    return rows


@pytest.mark.parametrize("nk,words", [((16, 11), 60000), ((32, 26), 60000), ((64, 57), 40000)])
def test_list_bler_calibration_matches_fig2(nk, words):
    pts = paper_points()[nk]
    # the paper's own points lie within 25% of the diagonal
    assert all(0.75 <= e / p <= 1.25 for p, e in pts)
    rows = calibration(synth.ebch(*nk), words, seed=101)
    assert check_list_bler_rows(nk, rows) >= 3


def check_list_bler_rows(nk, rows):
    """Every bin with at least 40 misses lies within 25 % (plus 4 sigma) of the diagonal, as the
    paper's own points do; returns the number of bins checked."""
    checked = 0
    for pred, emp, errs, cnt in rows:
        if errs < 40:
            continue
        checked += 1
        sd = np.sqrt(pred * (1 - pred) / cnt)
        assert abs(emp - pred) <= 0.25 * pred + 4 * sd, (nk, pred, emp, errs, cnt)
    return checked


def fig4_points():
    pts = {}
    for line in open(GOLDEN4):
        if line.startswith("#") or not line.strip():
            continue
        nk, b, p, e = line.split()
        pts.setdefault(tuple(int(x) for x in nk.split(",")), {})[int(b)] = (float(p), float(e))
    return pts


@pytest.mark.parametrize("nk,words", [((16, 11), 40000), ((32, 26), 30000), ((64, 57), 30000)])
def test_bitwise_so_calibration_matches_fig4(nk, words):
    """The bitwise soft output (eq. LLRi) binned by the predicted probability of a 1 reproduces
    the paper's Fig. 4 below 0.5: the same mean prediction per bin and the same empirical
    frequency.  Dropping the not-found term, taking the prior from L_Ch only, or a wrong
    list weighting moves these points by far more than the tolerance."""
    code = synth.ebch(*nk)
    llr, cw, _ = synth.component_words(code, 2.0, 202, np.arange(words))
    out = oracle.decode_component(code, llr, 4, 10 ** 5)
    check_bitwise_bins(nk, out["llr_app"], cw)


def check_bitwise_bins(nk, llr_app, cw):
    """Bits binned by the predicted probability of a 1 match the paper's Fig. 4 points below 0.5."""
    pts = fig4_points()[nk]
    p1 = 1.0 / (1.0 + np.exp(np.clip(llr_app, -700, 700)))
    bins = np.minimum((p1 * 20).astype(int), 19)
    for b, (pp, pe) in pts.items():
        sel = bins == b
        cnt = int(sel.sum())
        assert cnt >= 1000, (nk, b, cnt)
        pred = float(p1[sel].mean())
        emp = float(cw[sel].mean())
        sd = np.sqrt(emp * (1 - emp) / cnt)
        assert abs(pred - pp) <= 0.05 * pp + 5e-4, (nk, b, pred, pp)
        assert abs(emp - pe) <= 0.12 * pe + 4 * sd, (nk, b, emp, pe, cnt)
