"""Frames far below any usable Eb/N0 (-10 dB): almost every component word ends at a small query
cap without a full list, and every frame fails after its last half-iteration.  The plain,
batched and served forms against the oracle, frame by frame: success (all 0), half-iterations
(all 2 I_max), query sums and maxima, hard decisions bit-exact; L_APP within the parity bound."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import synth  # noqa: E402
from parity import compare_product  # noqa: E402

pytestmark = pytest.mark.gpu

NK = [(32, 26), (64, 57), (128, 120)]
L, CAP, ITERS, EBN0 = 4, 200, 2, -10.0


@pytest.fixture(scope="module")
def sg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    sg.lib()
    return sg


def check_failed(r, label):
    assert np.all(r["success"] == 0), label
    assert np.all(r["half_iters"].astype(np.int64) == 2 * ITERS), label


@pytest.mark.parametrize("nk", [(64, 57), (128, 120)])
@pytest.mark.parametrize("f32", [False, True])
def test_plain_fails_like_the_oracle(sg, nk, f32):
    import torch
    code = synth.ebch(*nk)
    llr = synth.product_frames(code, EBN0, 61, np.arange(8))[0]
    if f32:
        llr = llr.astype(np.float32).astype(np.float64)
    print(f"[gpu] plain {code.name}^2 at {EBN0} dB, cap {CAP}, f32={f32}", flush=True)
    g = sg.Code.from_hcols(code.n, code.k, code.hcols)
    x = torch.from_numpy(llr.astype(np.float32 if f32 else np.float64)).cuda()
    out = sg.sogrand_decode_product(g, x, list_max=L, query_cap=CAP, max_iter=ITERS, want_app=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    ref = oracle.decode_product(code, llr, L, CAP, ITERS, store_f32=f32, want_app=True, want_last_diag=True,
                                nthreads=8)
    check_failed(ref, "oracle")
    # most half-iterations have a word that ends at the cap
    assert np.mean(ref["sum_max_queries"] == 2 * ITERS * CAP) > 0.5
    compare_product(got, ref, f32=f32, label=f"plain {code.name}^2 at {EBN0} dB f32={f32}")


@pytest.fixture(scope="module")
def mixed():
    codes = [synth.ebch(*nk) for nk in NK]
    cidx, eb, offs, llr, cw = synth.mixed_product_frames(codes, EBN0, EBN0, 62, np.arange(30))
    llr = llr.astype(np.float32)
    ref = {}
    for c, code in enumerate(codes):
        sel = np.nonzero(cidx == c)[0]
        nn = code.n * code.n
        frames = np.stack([llr[o:o + nn] for o in offs[sel]]).astype(np.float64).reshape(-1, code.n, code.n)
        ref[c] = (sel, oracle.decode_product(code, frames, L, CAP, ITERS, store_f32=True, want_app=True,
                                             want_last_diag=True, nthreads=8))
        check_failed(ref[c][1], f"oracle {code.name}")
    return codes, cidx, offs, llr, ref


def gather(codes, c, sel, offs, flat):
    n = codes[c].n
    return np.stack([flat[o:o + n * n] for o in offs[sel]]).reshape(-1, n, n)


def test_batched_fails_like_the_oracle(sg, mixed):
    import torch
    codes, cidx, offs, llr, ref = mixed
    gcodes = [sg.Code.from_hcols(c.n, c.k, c.hcols) for c in codes]
    print(f"[gpu] batched, {cidx.size} mixed frames at {EBN0} dB, cap {CAP}", flush=True)
    out = sg.sogrand_decode_batched(gcodes, torch.from_numpy(cidx).cuda(), torch.from_numpy(offs).cuda(),
                                    torch.from_numpy(llr).cuda(), list_max=L, query_cap=CAP, max_iter=ITERS,
                                    want_app=True)
    torch.cuda.synchronize()
    b = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    assert int(b["status"][0]) == 0
    for c, (sel, r) in ref.items():
        g = dict(success=b["success"][sel], half_iters=b["half_iters"][sel], sum_queries=b["sum_queries"][sel],
                 sum_max_queries=b["sum_max_queries"][sel], hard=gather(codes, c, sel, offs, b["hard"]),
                 llr_app=gather(codes, c, sel, offs, b["llr_app"]))
        compare_product(g, r, f32=True, label=f"batched {codes[c].name}^2 at {EBN0} dB")


def test_served_fails_like_the_oracle(sg, mixed):
    codes, cidx, offs, llr, ref = mixed
    gcodes = [sg.Code.from_hcols(c.n, c.k, c.hcols) for c in codes]
    print(f"[gpu] served, {cidx.size} mixed frames at {EBN0} dB, cap {CAP}", flush=True)
    got, ids = {}, {}
    with sg.Server(64 << 20, list_max=L, query_cap=CAP, max_iter=ITERS, precision=sg.SOGRAND_F32,
                   export_app=True) as srv:
        pend = list(range(cidx.size))
        while pend or len(got) < cidx.size:
            while pend:
                f = pend[0]
                n = codes[cidx[f]].n
                rid = srv.submit(gcodes[cidx[f]], np.ascontiguousarray(llr[offs[f]:offs[f] + n * n]), tag=f)
                if rid is None:
                    break
                ids[rid] = f
                pend.pop(0)
            for r in srv.poll(max_results=64, timeout_ns=2_000_000):
                assert r["status"] == 0 and ids[r["request_id"]] == r["user_tag"]
                got[r["user_tag"]] = r
    for c, (sel, r) in ref.items():
        g = dict(success=np.array([got[f]["success"] for f in sel], np.uint8),
                 half_iters=np.array([got[f]["half_iters"] for f in sel]),
                 sum_queries=np.array([got[f]["queries"] for f in sel]),
                 hard=np.stack([got[f]["hard"] for f in sel]), llr_app=np.stack([got[f]["llr_app"] for f in sel]))
        compare_product(g, r, f32=True, label=f"served {codes[c].name}^2 at {EBN0} dB")
