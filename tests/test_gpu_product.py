"""GPU parity of block-turbo product decoding against the oracle (HIP kernels through the C ABI)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import synth  # noqa: E402
from parity import compare_product  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    sg.lib()
    return sg


def gpu_product(sg, code, llr, L, qcap, iters, f32=False, early_stop=True):
    import torch
    gcode = sg.Code.from_hcols(code.n, code.k, code.hcols)
    dt = torch.float32 if f32 else torch.float64
    x = torch.from_numpy(llr).to(dtype=dt, device="cuda").contiguous()
    out = sg.sogrand_decode_product(gcode, x, list_max=L, query_cap=qcap, max_iter=iters,
                                    early_stop=early_stop, want_app=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


CASES = [
    ((16, 11), 2.0, 40, 4, 1000, 4),
    ((32, 26), 3.0, 100, 4, 1000, 4),     # the small plain configuration: 100 frames, seed 0
    ((32, 26), 2.5, 60, 4, 1000, 4),
    ((64, 57), 2.5, 24, 4, 10000, 6),
    ((64, 57), 3.0, 24, 4, 10000, 6),
    ((128, 120), 3.0, 6, 4, 10000, 6),
    ((16, 7), 1.0, 30, 4, 1000, 4),
]


@pytest.mark.parametrize("nk,ebn0,frames,L,qcap,iters", CASES)
@pytest.mark.parametrize("f32", [False, True])
def test_product_parity(sg, nk, ebn0, frames, L, qcap, iters, f32):
    code = synth.ebch(*nk)
    seed = 0 if nk == (32, 26) and ebn0 == 3.0 else 40 + nk[0]
    llr, cw, _ = synth.product_frames(code, ebn0, seed, np.arange(frames))
    if f32:
        llr = llr.astype(np.float32).astype(np.float64)
    label = f"{code.name}^2 @{ebn0}dB f32={f32}"
    print(f"[gpu] product {label} frames={frames}", flush=True)
    g = gpu_product(sg, code, llr, L, qcap, iters, f32=f32)
    r = oracle.decode_product(code, llr, L, qcap, iters, store_f32=f32, want_app=True, want_last_diag=True, nthreads=8)
    compare_product(g, r, f32, label)
    print(f"[gpu]   ok; BLER {np.mean(np.any(g['hard'] != cw, axis=(1, 2))):.3f}", flush=True)


def hamming15():
    base = synth.ebch(16, 11)
    return synth.code_from_generator("Hamming[15,11]", base.G[:, :15], base.info_pos)


@pytest.mark.parametrize("which,ebn0,frames,qcap", [("hamming15", 2.5, 41, 1000), ("ebch8", 2.0, 50, 100)])
@pytest.mark.parametrize("f32", [False, True])
def test_product_parity_short_and_odd_codes(sg, which, ebn0, frames, qcap, f32):
    """Words of at most 32 bits go two to a wave.  With the odd length 15 and an odd frame count,
    pairs straddle frames and the last pair is half empty; Hamming[15,11] is also not an even code,
    so every weight is queried and the whole mass is the class.  [8,4] fills an eighth of a wave."""
    code = hamming15() if which == "hamming15" else synth.ebch(8, 4)
    llr, cw, _ = synth.product_frames(code, ebn0, 91, np.arange(frames))
    if f32:
        llr = llr.astype(np.float32).astype(np.float64)
    label = f"{code.name}^2 @{ebn0}dB f32={f32}"
    print(f"[gpu] product {label} frames={frames}", flush=True)
    g = gpu_product(sg, code, llr, 4, qcap, 4, f32=f32)
    r = oracle.decode_product(code, llr, 4, qcap, 4, store_f32=f32, want_app=True, want_last_diag=True, nthreads=8)
    compare_product(g, r, f32, label)
    assert r["half_iters"].max() > 2


@pytest.mark.parametrize("nk", [(32, 26), (64, 57)])
def test_product_parity_with_equal_and_nearly_equal_magnitudes(sg, nk):
    """Channel LLRs on a grid of 0.5 (many equal magnitudes, zeros of both signs), some moved by
    less than binary32 resolution, in frames that stop after the first row pass: the ranks must
    follow the binary64 magnitudes, ties by bit index.  (Later half-iterations add a-priori LLRs
    whose last bits differ between the two implementations; on such a grid, magnitudes that are
    equal on one side can then differ by an ulp on the other, and the tie rule would order them
    differently.  With unquantised channel noise such coincidences have no measurable chance.)"""
    code = synth.ebch(*nk)
    llr, _, _ = synth.product_frames(code, 6.0, 5, np.arange(40))
    llr = np.round(llr * 2) / 2
    llr[0, 0, :] = 0.0
    llr[1, 0, :] = -0.0
    nudge = np.random.default_rng(1).integers(0, 3, size=llr.shape) * 2.0 ** -40   # below binary32 resolution
    llr = llr + np.sign(llr) * nudge
    r = oracle.decode_product(code, llr, 4, 3000, 4, want_app=True, want_last_diag=True, nthreads=8)
    one = np.nonzero(r["half_iters"] == 1)[0]
    assert one.size >= 30
    llr = llr[one]
    r = {k: v[one] for k, v in r.items() if v is not None}
    print(f"[gpu] product ties {code.name}^2, {one.size} frames", flush=True)
    g = gpu_product(sg, code, llr, 4, 3000, 4)
    compare_product(g, r, label=f"ties {code.name}")


def test_product_without_early_stop(sg):
    code = synth.ebch(32, 26)
    llr, _, _ = synth.product_frames(code, 3.0, 9, np.arange(20))
    g = gpu_product(sg, code, llr, 4, 1000, 3, early_stop=False)
    r = oracle.decode_product(code, llr, 4, 1000, 3, early_stop=False, want_app=True, want_last_diag=True)
    compare_product(g, r, label="no early stop")
    assert np.all(g["half_iters"] == 6)


def test_product_ragged_frame_counts(sg):
    code = synth.ebch(64, 57)
    for F in (1, 3, 5):
        llr, _, _ = synth.product_frames(code, 3.0, 77 + F, np.arange(F))
        g = gpu_product(sg, code, llr, 4, 2000, 3)
        r = oracle.decode_product(code, llr, 4, 2000, 3, want_app=True, want_last_diag=True)
        compare_product(g, r, label=f"F={F}")


def test_full_size_product_workload_sampled(sg):
    """The [64,57]^2 workload at full size (1e4 frames per Eb/N0, L = 4, cap 1e4, 6 iterations),
    decoded in the launch configuration the benchmark times; sampled frames vs the oracle."""
    import torch
    code = synth.ebch(64, 57)
    gcode = sg.Code.ebch(64, 57)
    rng = np.random.default_rng(1)
    for snr, seed in ((2.5, 1), (3.0, 2), (3.5, 3)):
        for f32 in (False, True):
            print(f"[gpu] full product {snr} dB f32={f32}", flush=True)
            llr, cw, _ = synth.product_frames(code, snr, seed, np.arange(10000))
            dt = torch.float32 if f32 else torch.float64
            x = torch.from_numpy(llr).to(dtype=dt, device="cuda")
            out = sg.sogrand_decode_product(gcode, x, list_max=4, query_cap=10000, max_iter=6, want_app=False)
            torch.cuda.synchronize()
            sample = np.sort(rng.choice(10000, size=12, replace=False))
            g = {k: v.cpu().numpy()[sample] for k, v in out.items() if v is not None}
            ls = llr[sample].astype(np.float32).astype(np.float64) if f32 else llr[sample]
            r = oracle.decode_product(code, ls, 4, 10000, 6, store_f32=f32, nthreads=8)
            for key in ("success", "half_iters", "sum_queries", "sum_max_queries", "hard"):
                np.testing.assert_array_equal(g[key].astype(np.int64), r[key].astype(np.int64), err_msg=key)
            hard = out["hard"].cpu().numpy()
            bler = np.mean(np.any(hard != cw, axis=(1, 2)))
            print(f"[gpu]   BLER {bler:.4g}; mean half-iters {out['half_iters'].double().mean().item():.2f}",
                  flush=True)
            del x, out


@pytest.mark.parametrize("f32", [False, True])
def test_product_parity_rician(sg, f32):
    """[32,26]^2 over block Rician fading with QPSK (N_c = 256, t = 2, K = 8) with the paper's fading
    settings (alpha 0.5, I_max 20, list-BLER stop 1e-4): deep fades give the decoder inputs far
    from the AWGN ones."""
    import torch
    code = synth.ebch(32, 26)
    llr, cw, _ = synth.rician_product_frames(code, 6.0, 8.0, 256, 31, np.arange(60))
    if f32:
        llr = llr.astype(np.float32).astype(np.float64)
    label = f"rician {code.name}^2 f32={f32}"
    print(f"[gpu] product {label}", flush=True)
    gcode = sg.Code.from_hcols(code.n, code.k, code.hcols)
    x = torch.from_numpy(llr).to(dtype=torch.float32 if f32 else torch.float64, device="cuda").contiguous()
    out = sg.sogrand_decode_product(gcode, x, list_max=4, query_cap=10000, max_iter=20, want_app=True,
                                    list_bler_stop=1e-4)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    r = oracle.decode_product(code, llr, 4, 10000, 20, store_f32=f32, want_app=True, pstop=1e-4, want_last_diag=True, nthreads=8)
    compare_product(g, r, f32, label)
    assert r["half_iters"].max() > 2


def test_full_size_batched_workload_sampled(sg):
    """The default benchmark line's form: all 3e4 [64,57]^2 frames in one persistent launch with the
    default launch shape and binary32 storage.  Every frame equals the plain path's decode, and
    sampled frames equal the oracle's."""
    import torch
    code = synth.ebch(64, 57)
    gcode = sg.Code.ebch(64, 57)
    parts = [synth.product_frames(code, snr, seed, np.arange(10000))[0] for snr, seed in ((2.5, 1), (3.0, 2), (3.5, 3))]
    llr = np.concatenate(parts)
    F = llr.shape[0]
    x = torch.from_numpy(llr).to(dtype=torch.float32, device="cuda")
    print("[gpu] full batched [64,57]^2 f32", flush=True)
    fc = torch.zeros(F, dtype=torch.uint8, device="cuda")
    fo = torch.arange(F, dtype=torch.int64, device="cuda") * (64 * 64)
    b = sg.sogrand_decode_batched([gcode], fc, fo, x.view(-1), list_max=4, query_cap=10000, max_iter=6)
    p = sg.sogrand_decode_product(gcode, x, list_max=4, query_cap=10000, max_iter=6)
    torch.cuda.synchronize()
    assert int(b["status"].item()) == 0
    for key in ("success", "half_iters", "sum_queries", "sum_max_queries"):
        assert torch.equal(b[key].to(torch.int64), p[key].to(torch.int64)), key
    assert torch.equal(b["hard"].view(F, 64, 64), p["hard"])
    rng = np.random.default_rng(2)
    sample = np.sort(rng.choice(F, size=24, replace=False))
    r = oracle.decode_product(code, llr[sample].astype(np.float32).astype(np.float64), 4, 10000, 6,
                              store_f32=True, nthreads=8)
    for key in ("success", "half_iters", "sum_queries", "sum_max_queries"):
        np.testing.assert_array_equal(b[key].cpu().numpy()[sample].astype(np.int64), r[key].astype(np.int64),
                                      err_msg=key)
    np.testing.assert_array_equal(b["hard"].view(F, 64, 64).cpu().numpy()[sample], r["hard"])
