"""The batched and served forms at the operating point of the mixed-stream and serving
workloads (L = 4, query cap 10^5, 6 iterations, alpha 0.5, binary32 storage), frame by frame
against the oracle: success, half-iterations, query sums (and per-half maxima for the batched
form) and hard decisions bit-exact, L_APP within the binary32 bound.

Frames: the first 60 frames of the mixed stream ([32,26]^2, [64,57]^2, [128,120]^2 eBCH, Eb/N0
uniform in [2, 4] dB, seed 4), plus 6 frames of a low-rate even [32,8] component code.  The
eBCH words never come near the cap at these settings (with n - k <= 8 a list of four is found
within a few thousand queries); the [32,8] words (n - k = 24) reach it in every half-iteration,
so the cap path runs in the same launch and server as the rest.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import synth  # noqa: E402
from codes import small_code  # noqa: E402
from parity import compare_product  # noqa: E402

pytestmark = pytest.mark.gpu

NK = [(32, 26), (64, 57), (128, 120)]
L, CAP, ITERS = 4, 100000, 6


@pytest.fixture(scope="module")
def sg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    sg.lib()
    return sg


@pytest.fixture(scope="module")
def case():
    """Frames (binary32-rounded), their layout, and the oracle's decode of every frame."""
    codes = [synth.ebch(*nk) for nk in NK]
    cidx, eb, offs, llr, cw = synth.mixed_product_frames(codes, 2.0, 4.0, 4, np.arange(60))
    low = small_code(32, 8, True, 5)
    lr, _, _ = synth.product_frames(low, 2.5, 41, np.arange(6))
    codes.append(low)
    base = llr.shape[0]
    llr = np.concatenate([llr, lr.reshape(-1)]).astype(np.float32)
    cidx = np.concatenate([cidx, np.full(6, 3, np.uint8)])
    offs = np.concatenate([offs, base + np.arange(6, dtype=np.int64) * 32 * 32])
    ref = {}
    for c, code in enumerate(codes):
        sel = np.nonzero(cidx == c)[0]
        nn = code.n * code.n
        frames = np.stack([llr[o:o + nn] for o in offs[sel]]).astype(np.float64).reshape(-1, code.n, code.n)
        ref[c] = (sel, oracle.decode_product(code, frames, L, CAP, ITERS, store_f32=True, want_app=True,
                                             want_last_diag=True, nthreads=8))
    # the low-rate frames reach the cap in every half-iteration
    r3 = ref[3][1]
    assert np.all(r3["sum_max_queries"] == r3["half_iters"].astype(np.int64) * CAP)
    return codes, cidx, offs, llr, ref


def gather(codes, c, sel, offs, flat):
    """Frames sel of code c, (len(sel), n, n), from a flat buffer laid out by offs."""
    n = codes[c].n
    return np.stack([flat[o:o + n * n] for o in offs[sel]]).reshape(-1, n, n)


def test_batched_matches_oracle_at_operating_point(sg, case):
    import torch
    codes, cidx, offs, llr, ref = case
    gcodes = [sg.Code.from_hcols(c.n, c.k, c.hcols) for c in codes]
    print(f"[gpu] batched operating point: {cidx.size} frames, cap {CAP}", flush=True)
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
        compare_product(g, r, f32=True, label=f"batched {codes[c].name}^2 at the operating point")


def test_served_matches_oracle_at_operating_point(sg, case):
    codes, cidx, offs, llr, ref = case
    gcodes = [sg.Code.from_hcols(c.n, c.k, c.hcols) for c in codes]
    print(f"[gpu] served operating point: {cidx.size} frames, cap {CAP}", flush=True)
    got, ids = {}, {}
    with sg.Server(256 << 20, list_max=L, query_cap=CAP, max_iter=ITERS, precision=sg.SOGRAND_F32,
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
                if len(ids) % 7 == 0:
                    break   # let earlier frames get going before the next ones join
            for r in srv.poll(max_results=64, timeout_ns=2_000_000):
                assert r["status"] == 0 and ids[r["request_id"]] == r["user_tag"]
                got[r["user_tag"]] = r
    for c, (sel, r) in ref.items():
        g = dict(success=np.array([got[f]["success"] for f in sel], np.uint8),
                 half_iters=np.array([got[f]["half_iters"] for f in sel]),
                 sum_queries=np.array([got[f]["queries"] for f in sel]),
                 hard=np.stack([got[f]["hard"] for f in sel]), llr_app=np.stack([got[f]["llr_app"] for f in sel]))
        compare_product(g, r, f32=True, label=f"served {codes[c].name}^2 at the operating point")


def test_plain_matches_oracle_on_cap_reaching_frames(sg, case):
    """The plain path on the [32,8] frames whose every word reaches the cap (binary32 and binary64)."""
    import torch
    codes, cidx, offs, llr, ref = case
    sel, r32 = ref[3]
    code = codes[3]
    frames = gather(codes, 3, sel, offs, llr)
    g = sg.Code.from_hcols(code.n, code.k, code.hcols)
    for f32 in (True, False):
        x = torch.from_numpy(frames.astype(np.float32 if f32 else np.float64)).cuda()
        out = sg.sogrand_decode_product(g, x, list_max=L, query_cap=CAP, max_iter=ITERS, want_app=True)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
        r = r32 if f32 else oracle.decode_product(code, frames.astype(np.float64), L, CAP, ITERS, want_app=True,
                                                  want_last_diag=True, nthreads=8)
        compare_product(got, r, f32=f32, label=f"plain {code.name}^2 cap-reaching f32={f32}")
