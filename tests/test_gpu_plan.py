"""Plans: a product or QC-GLDPC decode recorded once as a HIP graph.  Every replay, with the
program's own device work and synchronisations between replays, gives exactly what the eager
call gives on the frames that the input buffer holds at that time."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

KEYS = ("hard", "success", "half_iters", "sum_queries", "sum_max_queries", "llr_app")


@pytest.fixture(scope="module")
def sg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    sg.lib()
    return sg


def frame_sets(nk, gldpc, ebn0, F, seeds):
    code = synth.ebch(*nk)
    if gldpc:
        g = synth.gldpc(code)
        return code, [synth.gldpc_frames(g, ebn0, s, np.arange(F))[0] for s in seeds]
    return code, [synth.product_frames(code, ebn0, s, np.arange(F))[0] for s in seeds]


# (code, gldpc, Eb/N0, frames, cap, I_max, f32): the small product case, the paper's I_max = 20
# (81 launches), binary32 [64,57]^2 frames and QC-GLDPC frames of [32,26] components
CASES = [((32, 26), False, 3.0, 100, 1000, 4, False),
         ((32, 26), False, 2.5, 37, 1000, 20, False),
         ((64, 57), False, 3.0, 200, 10000, 6, True),
         ((32, 26), True, 2.25, 20, 3000, 8, True)]


@pytest.mark.parametrize("nk,gldpc,ebn0,F,qcap,iters,f32", CASES)
def test_plan_replays_equal_eager_decodes(sg, nk, gldpc, ebn0, F, qcap, iters, f32):
    import torch
    code, sets = frame_sets(nk, gldpc, ebn0, F, seeds=[5, 6, 5])
    g = sg.Code.from_hcols(code.n, code.k, code.hcols)
    dt = torch.float32 if f32 else torch.float64
    alpha = 0.6 if gldpc else 0.5
    x = torch.empty((F, code.n, code.n), dtype=dt, device="cuda")
    x.copy_(torch.from_numpy(sets[0]).to(dt))
    print(f"[gpu] plan {code.name} gldpc={gldpc} F={F} I_max={iters} f32={f32}", flush=True)
    plan = sg.Plan(g, x, list_max=4, query_cap=qcap, max_iter=iters, alpha=alpha, want_app=True, gldpc=gldpc)
    eager = sg.sogrand_decode_gldpc if gldpc else sg.sogrand_decode_product
    try:
        for r, llr in enumerate(sets):
            x.copy_(torch.from_numpy(llr).to(dt))
            for v in plan.outputs.values():     # device work of the program's own between replays
                v.fill_(0x5A if v.dtype == torch.uint8 else 3)
            torch.cuda.synchronize()
            got = plan.launch()
            torch.cuda.synchronize()
            ref = eager(g, x.clone(), list_max=4, query_cap=qcap, max_iter=iters, alpha=alpha, want_app=True)
            torch.cuda.synchronize()
            for key in KEYS:
                assert torch.equal(got[key], ref[key]), (r, key)
    finally:
        plan.close()
