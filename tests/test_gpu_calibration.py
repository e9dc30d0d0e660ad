"""The soft-output calibration of the paper's Figs. 2 and 4 at scale, decoded on the GPU.

Millions of component words at 2 dB go through sogrand_decode_component.  On them:
* SOGRAND's predicted list-BLER (eq. app_approxlist, L = 4) stays on the diagonal down to bins the
  oracle-sized tests cannot reach, a large-scale check of the parity-class reading of Corollary 1;
* Forney's approximation (eq. missingterm) over a list of 5, formed from the GPU's list APPs,
  under-predicts the list-BLER of the first 4 as the paper's dashed Fig. 2 curves do;
* the bitwise soft output (eq. LLRi) reproduces Fig. 4.
The list APPs are tied to the oracle: their ratios equal the oracle's Forney weights from the
likelihoods of the GPU's own lists, and a sample of words decodes to the oracle's lists exactly.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import synth  # noqa: E402
from test_oracle_calibration import check_bitwise_bins, check_list_bler_rows  # noqa: E402
from test_oracle_forney import binned, check_forney_curve, in_first  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    sg.lib()
    return sg


def gpu_list(sg, gcode, x, L):
    import torch
    out = sg.sogrand_decode_component(gcode, x, list_max=L, query_cap=10 ** 5, found_z=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def table(name, rows):
    for pred, emp, errs, cnt in rows:
        print(f"[gpu]   {name} pred {pred:.4g} emp {emp:.4g} misses {errs} words {cnt}", flush=True)


@pytest.mark.parametrize("nk,words", [((16, 11), 2_000_000), ((32, 26), 2_000_000), ((64, 57), 1_000_000)])
def test_calibration_at_scale(sg, nk, words):
    import torch
    print(f"[gpu] calibration eBCH{nk} at 2 dB, {words} words", flush=True)
    code = synth.ebch(*nk)
    gcode = sg.Code.ebch(*nk)
    llr, cw, _ = synth.component_words(code, 2.0, 301, np.arange(words))
    x = torch.from_numpy(llr).to("cuda")

    g4 = gpu_list(sg, gcode, x, 4)
    hit4 = in_first(llr, cw, g4["found_z"], g4["n_found"].astype(np.int64), 4)
    rows = binned(g4["p_notfound"], hit4)
    table("SOGRAND L=4", rows)
    assert check_list_bler_rows(nk, rows) >= 5
    check_bitwise_bins(nk, g4["llr_app"][:200_000], cw[:200_000])

    g5 = gpu_list(sg, gcode, x, 5)
    nf = g5["n_found"].astype(np.int64)
    valid = np.arange(5)[None, :] < nf[:, None]
    pf = np.where(valid, g5["p_found"], 0.0)
    forney = pf / pf.sum(axis=1, keepdims=True)
    ref = oracle.forney_app(llr, g5["found_z"], nf)
    np.testing.assert_allclose(forney, ref, rtol=1e-9, atol=1e-15)
    pred = np.maximum(1.0 - forney[:, :4].sum(axis=1), 0.0)
    rows5 = binned(pred, in_first(llr, cw, g5["found_z"], nf, 4))
    table("Forney L=5", rows5)
    assert check_forney_curve(nk, rows5, factor=1.6) >= 4

    sample = np.arange(0, words, words // 2000)
    want = oracle.decode_component(code, llr[sample], 5, 10 ** 5, want_z=True)
    np.testing.assert_array_equal(g5["n_queries"][sample], want["n_queries"].astype(np.int32))
    np.testing.assert_array_equal(nf[sample], want["n_found"])
    np.testing.assert_array_equal(g5["found_z"][sample], want["found_z"])
    del x
