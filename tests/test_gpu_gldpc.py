"""GPU parity of QC-GLDPC decoding (sogrand_decode_gldpc) against the oracle."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import synth  # noqa: E402
from test_gpu_product import compare_product  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    sg.lib()
    return sg


def gpu_gldpc(sg, code, llr, L, qcap, iters, alpha, f32=False, stop=0.0):
    import torch
    gcode = sg.Code.from_hcols(code.n, code.k, code.hcols)
    dt = torch.float32 if f32 else torch.float64
    x = torch.from_numpy(llr).to(dtype=dt, device="cuda").contiguous()
    out = sg.sogrand_decode_gldpc(gcode, x, list_max=L, query_cap=qcap, max_iter=iters, alpha=alpha,
                                  want_app=True, list_bler_stop=stop)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


# (component, Eb/N0, frames, L, cap, I_max, alpha, stop): the paper's GLDPC settings (alpha 0.6,
# I_max 20, stop 1e-5) at its waterfall, the same without the stop, and a second component length
CASES = [
    ((32, 26), 2.0, 60, 4, 10000, 20, 0.6, 1e-5),
    ((32, 26), 2.25, 60, 4, 10000, 20, 0.6, 0.0),
    ((32, 26), 2.5, 37, 4, 3000, 8, 0.5, 0.0),      # a ragged frame count
    ((16, 11), 2.0, 50, 4, 1000, 10, 0.6, 0.0),
]


@pytest.mark.parametrize("nk,ebn0,frames,L,qcap,iters,alpha,stop", CASES)
@pytest.mark.parametrize("f32", [False, True])
def test_gldpc_parity(sg, nk, ebn0, frames, L, qcap, iters, alpha, stop, f32):
    code = synth.ebch(*nk)
    g = synth.gldpc(code)
    llr, cw, _ = synth.gldpc_frames(g, ebn0, 70 + nk[0], np.arange(frames))
    if f32:
        llr = llr.astype(np.float32).astype(np.float64)
    label = f"GLDPC[{code.name}] @{ebn0}dB f32={f32} stop={stop}"
    print(f"[gpu] gldpc {label} frames={frames}", flush=True)
    got = gpu_gldpc(sg, code, llr, L, qcap, iters, alpha, f32=f32, stop=stop)
    ref = oracle.decode_gldpc(code, llr, L, qcap, iters, alpha, store_f32=f32, want_app=True, pstop=stop,
                              nthreads=8)
    worst = compare_product(got, ref, f32, label)
    assert ref["half_iters"].max() > 2
    print(f"[gpu]   ok; BLER {np.mean(np.any(got['hard'] != cw, axis=(1, 2))):.3f}, worst rel dL {worst:.2e}",
          flush=True)


def test_gldpc_empty_and_bad_shape(sg):
    import torch
    code = synth.ebch(32, 26)
    gcode = sg.Code.from_hcols(code.n, code.k, code.hcols)
    out = sg.sogrand_decode_gldpc(gcode, torch.zeros((0, 32, 32), dtype=torch.float64, device="cuda"))
    assert out["hard"].shape == (0, 32, 32)
    with pytest.raises(ValueError):
        sg.sogrand_decode_gldpc(gcode, torch.zeros((2, 32, 16), dtype=torch.float64, device="cuda"))


def test_full_size_gldpc_workload_sampled(sg):
    """The QC-GLDPC benchmark workload at full size (1e4 frames at each of 2.0/2.25/2.5 dB, alpha 0.6,
    I_max 20, stop 1e-5, binary32 storage) in the launch the benchmark times; sampled frames vs the
    oracle."""
    import torch
    code = synth.ebch(32, 26)
    g = synth.gldpc(code)
    gcode = sg.Code.ebch(32, 26)
    rng = np.random.default_rng(3)
    for snr, seed in ((2.0, 11), (2.25, 12), (2.5, 13)):
        print(f"[gpu] full gldpc {snr} dB", flush=True)
        llr, cw, _ = synth.gldpc_frames(g, snr, seed, np.arange(10000))
        x = torch.from_numpy(llr).to(dtype=torch.float32, device="cuda")
        out = sg.sogrand_decode_gldpc(gcode, x, list_max=4, query_cap=10000, max_iter=20, alpha=0.6,
                                      list_bler_stop=1e-5)
        torch.cuda.synchronize()
        sample = np.sort(rng.choice(10000, size=20, replace=False))
        got = {k: v.cpu().numpy()[sample] for k, v in out.items() if v is not None}
        ref = oracle.decode_gldpc(code, llr[sample].astype(np.float32).astype(np.float64), 4, 10000, 20, 0.6,
                                  store_f32=True, pstop=1e-5, nthreads=8)
        for key in ("success", "half_iters", "sum_queries", "sum_max_queries", "hard"):
            np.testing.assert_array_equal(got[key].astype(np.int64), ref[key].astype(np.int64), err_msg=key)
        del x, out
