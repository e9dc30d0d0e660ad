"""GPU parity of component SOGRAND decoding (HIP kernels through the C ABI) against the oracle."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import synth  # noqa: E402
from codes import small_code  # noqa: E402
from parity import compare_component  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    sg.lib()
    return sg


def hamming15():
    base = synth.ebch(16, 11)
    return synth.code_from_generator("Hamming[15,11]", base.G[:, :15], base.info_pos)


def run_pair(sg, ref_code, llr, L, qcap, f32=False, label=""):
    import torch
    code = sg.Code.from_hcols(ref_code.n, ref_code.k, ref_code.hcols)
    dt = torch.float32 if f32 else torch.float64
    x = torch.from_numpy(llr).to(dtype=dt, device="cuda").contiguous()
    print(f"[gpu] component {label} words={llr.shape[0]} L={L} cap={qcap} f32={f32}", flush=True)
    out = sg.sogrand_decode_component(code, x, list_max=L, query_cap=qcap, found_z=True)
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    llr_ref = llr.astype(np.float32).astype(np.float64) if f32 else llr
    ref = oracle.decode_component(ref_code, llr_ref, L, qcap, want_z=True, want_diag=True)
    return compare_component(g, ref, f32=f32, label=label)


CODES = [(8, 4), (16, 11), (32, 26), (64, 57), (128, 120), (16, 7)]


@pytest.mark.parametrize("nk", CODES)
@pytest.mark.parametrize("ebn0", [1.0, 3.0, 5.0])
def test_component_parity_f64(sg, nk, ebn0):
    code = synth.ebch(*nk)
    llr, _, _ = synth.component_words(code, ebn0, 1000 + nk[0], np.arange(203))
    for L, qcap in [(1, 1000), (4, 1000), (4, 37), (3, 5000)]:
        run_pair(sg, code, llr, L, qcap, label=f"{code.name}@{ebn0}dB")


@pytest.mark.parametrize("nk", [(32, 26), (64, 57), (128, 120)])
def test_component_parity_f32(sg, nk):
    code = synth.ebch(*nk)
    llr, _, _ = synth.component_words(code, 3.0, 7 + nk[0], np.arange(401))
    for L, qcap in [(1, 1000), (4, 10000)]:
        run_pair(sg, code, llr, L, qcap, f32=True, label=f"{code.name} f32")


def test_non_even_code(sg):
    code = hamming15()
    llr, _, _ = synth.component_words(code, 2.0, 3, np.arange(150))
    run_pair(sg, code, llr, 4, 2000, label="Hamming[15,11]")


def test_edge_cases(sg):
    code = synth.ebch(8, 4)
    llr, _, _ = synth.component_words(code, 0.0, 5, np.arange(9))
    run_pair(sg, code, llr, 16, 1 << 20, label="[8,4] exhaustive class, L=16")
    run_pair(sg, code, llr, 4, 1, label="[8,4] cap 1")
    c64 = synth.ebch(64, 57)
    ties = np.round(synth.component_words(c64, 2.0, 6, np.arange(40))[0] * 2) / 2   # many equal |LLR|
    ties[0] = 0.0
    ties[1] = -0.0
    ties[2, ::2] = 3.0
    run_pair(sg, c64, ties, 4, 3000, label="ties and zeros")
    big = np.where(synth.component_words(c64, 3.0, 8, np.arange(12))[0] < 0, -40.0, 40.0)
    run_pair(sg, c64, big, 4, 1000, label="saturated")
    for W in (1, 2, 3, 5, 63, 65):
        llr, _, _ = synth.component_words(c64, 2.5, 100 + W, np.arange(W))
        run_pair(sg, c64, llr, 4, 500, label=f"ragged {W}")


@pytest.mark.parametrize("n,k,even", [(8, 3, True), (16, 3, True), (12, 3, False)])
def test_exhausted_class_gives_exact_app(sg, n, k, even):
    """A list longer than the codebook runs the search through the whole class: every
    codeword is found, the not-found mass is exactly zero, and eq. (LLRi) is the exact bitwise
    APP LLR, summed here over the codebook (within 1e-12 relative)."""
    code = small_code(n, k, even, 100 + n)
    assert code.is_even == even
    llr, _, _ = synth.component_words(code, 0.5, 31 + n, np.arange(70))
    L, cap = (1 << k) + 1, 1 << (n - 1 if even else n)
    run_pair(sg, code, llr, L, cap, label=f"{code.name} exhausted class")
    import torch
    gcode = sg.Code.from_hcols(code.n, code.k, code.hcols)
    out = sg.sogrand_decode_component(gcode, torch.from_numpy(llr).cuda(), list_max=L, query_cap=cap)
    torch.cuda.synchronize()
    assert np.all(out["n_queries"].cpu().numpy() == cap)
    assert np.all(out["n_found"].cpu().numpy() == 1 << k)
    assert np.all(out["p_notfound"].cpu().numpy() == 0.0)
    msgs = ((np.arange(1 << k)[:, None] >> np.arange(k)) & 1).astype(np.int64)
    cb = ((msgs @ code.G.astype(np.int64)) % 2).astype(np.float64)
    s = (llr[:, None, :] * (1.0 - 2.0 * cb)).sum(-1) / 2.0
    w = np.exp(s - s.max(1, keepdims=True))
    exact = np.log((w[:, :, None] * (cb == 0)).sum(1)) - np.log((w[:, :, None] * (cb == 1)).sum(1))
    got = out["llr_app"].cpu().numpy()
    err = np.abs(got - exact) / np.maximum(1.0, np.abs(exact))
    print(f"[gpu]   worst relative difference from the codebook APP {err.max():.2e}", flush=True)
    assert err.max() <= 1e-12


@pytest.mark.parametrize("nk", [(32, 26), (64, 57), (128, 120)])
def test_nearly_equal_magnitudes(sg, nk):
    """Magnitudes on a grid of 0.5, some moved by less than binary32 resolution: equal binary32
    keys whose binary64 values differ must be ranked by the binary64 values."""
    code = synth.ebch(*nk)
    llr = np.round(synth.component_words(code, 2.0, 9, np.arange(60))[0] * 2) / 2
    nudge = np.random.default_rng(2).integers(0, 4, size=llr.shape) * 2.0 ** -41
    llr = llr + np.where(llr < 0, -1.0, 1.0) * nudge
    run_pair(sg, code, llr, 4, 3000, label=f"{code.name} near-equal magnitudes")


def test_empty_batch_is_a_no_op(sg):
    import torch
    code = sg.Code.ebch(32, 26)
    x = torch.empty((0, 32), dtype=torch.float64, device="cuda")
    out = sg.sogrand_decode_component(code, x)
    torch.cuda.synchronize()
    assert out["llr_app"].shape == (0, 32)


def test_full_size_component_workload_sampled(sg):
    """2^20 [128,120] words at 4 dB (L = 1 and 4, cap 1e5) in one launch; sampled words vs the oracle."""
    import torch
    code = synth.ebch(128, 120)
    gcode = sg.Code.ebch(128, 120)
    nw = 1 << 20
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(nw, size=600, replace=False))
    llr_s, _, _ = synth.component_words(code, 4.0, 5, sample)
    for L in (1, 4):
        print(f"[gpu] full component 2^20 L={L}", flush=True)
        x = torch.empty((nw, 128), dtype=torch.float32, device="cuda")
        chunk = 1 << 17
        for s in range(0, nw, chunk):
            llr, _, _ = synth.component_words(code, 4.0, 5, np.arange(s, s + chunk))
            x[s:s + chunk] = torch.from_numpy(llr.astype(np.float32))
        out = sg.sogrand_decode_component(gcode, x, list_max=L, query_cap=100000, found_z=False)
        torch.cuda.synchronize()
        idx = torch.from_numpy(sample).cuda()
        g = {k: v[idx].cpu().numpy() for k, v in out.items() if v is not None}
        g["found_z"] = None
        ref = oracle.decode_component(code, llr_s.astype(np.float32).astype(np.float64), L, 100000,
                                      want_z=True, want_diag=True)
        compare_component(g, ref, f32=True, label=f"2^20 words L={L}")
        nq = out["n_queries"].double()
        print(f"[gpu]   mean queries {nq.mean().item():.1f} max {nq.max().item():.0f}", flush=True)
        del x, out
