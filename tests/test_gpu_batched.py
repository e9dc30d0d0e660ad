"""Batched persistent decoding of mixed-code product frames: identical per-frame results to the
plain path, parity with the oracle on a sample, independence of the launch shape, and the
handling of invalid frame descriptors."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

NK = [(32, 26), (64, 57), (128, 120)]


@pytest.fixture(scope="module")
def sg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    sg.lib()
    return sg


def mixed(F, seed, lo=2.0, hi=4.0, nks=NK):
    codes = [synth.ebch(*nk) for nk in nks]
    cidx, eb, offs, llr, cw = synth.mixed_product_frames(codes, lo, hi, seed, np.arange(F))
    return codes, cidx, eb, offs, llr, cw


def handle(sg, code):
    """The library's code object for a synth code, built from its H columns."""
    return sg.Code.from_hcols(code.n, code.k, code.hcols)


def run_batched(sg, codes, cidx, offs, llr, f32=False, sched=None, L=4, qcap=10000, iters=6):
    import torch
    gcodes = [handle(sg, c) for c in codes]
    dt = torch.float32 if f32 else torch.float64
    x = torch.from_numpy(llr).to(dtype=dt, device="cuda")
    fc = torch.from_numpy(cidx).cuda()
    fo = torch.from_numpy(offs).cuda()
    out = sg.sogrand_decode_batched(gcodes, fc, fo, x, list_max=L, query_cap=qcap, max_iter=iters, sched_=sched)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def run_plain_per_code(sg, codes, cidx, offs, llr, f32=False, L=4, qcap=10000, iters=6):
    import torch
    F = cidx.shape[0]
    res = dict(success=np.zeros(F, np.uint8), half_iters=np.zeros(F, np.int64), sum_queries=np.zeros(F, np.int64),
               sum_max_queries=np.zeros(F, np.int64), hard=np.zeros(llr.shape, np.uint8))
    dt = torch.float32 if f32 else torch.float64
    for c, code in enumerate(codes):
        sel = np.nonzero(cidx == c)[0]
        if sel.size == 0:
            continue
        nn = code.n * code.n
        frames = np.stack([llr[o:o + nn] for o in offs[sel]]).reshape(-1, code.n, code.n)
        g = handle(sg, code)
        out = sg.sogrand_decode_product(g, torch.from_numpy(frames).to(dtype=dt, device="cuda"), list_max=L,
                                        query_cap=qcap, max_iter=iters)
        torch.cuda.synchronize()
        for key in ("success", "half_iters", "sum_queries", "sum_max_queries"):
            res[key][sel] = out[key].cpu().numpy()
        hard = out["hard"].cpu().numpy().reshape(-1, nn)
        for j, o in enumerate(offs[sel]):
            res["hard"][o:o + nn] = hard[j]
    return res


@pytest.mark.parametrize("f32", [False, True])
def test_batched_equals_plain_per_frame(sg, f32):
    codes, cidx, eb, offs, llr, cw = mixed(600, seed=4)
    print(f"[gpu] batched vs plain, 600 mixed frames, f32={f32}", flush=True)
    b = run_batched(sg, codes, cidx, offs, llr, f32=f32)
    p = run_plain_per_code(sg, codes, cidx, offs, llr, f32=f32)
    assert int(b["status"][0]) == 0
    for key in ("success", "half_iters", "sum_queries", "sum_max_queries"):
        np.testing.assert_array_equal(b[key].astype(np.int64), p[key].astype(np.int64), err_msg=key)
    np.testing.assert_array_equal(b["hard"], p["hard"])


@pytest.mark.parametrize("with64", [True, False])
def test_batched_equals_plain_for_short_and_odd_codes(sg, with64):
    """Non-even Hamming[15,11] (odd length) and [8,4] frames, with [64,57] frames (one word per wave)
    or without them (two words per wave), in one launch: equal to the plain path per code and, on a
    sample, to the oracle."""
    base = synth.ebch(16, 11)
    codes = [synth.code_from_generator("Hamming[15,11]", base.G[:, :15], base.info_pos), synth.ebch(8, 4)]
    if with64:
        codes.append(synth.ebch(64, 57))
    cidx, eb, offs, llr, cw = synth.mixed_product_frames(codes, 2.0, 3.5, 13, np.arange(300))
    print(f"[gpu] batched, Hamming[15,11] + [8,4]{' + [64,57]' if with64 else ''}, 300 frames", flush=True)
    b = run_batched(sg, codes, cidx, offs, llr, qcap=3000, iters=4)
    p = run_plain_per_code(sg, codes, cidx, offs, llr, qcap=3000, iters=4)
    assert int(b["status"][0]) == 0
    for key in ("success", "half_iters", "sum_queries", "sum_max_queries"):
        np.testing.assert_array_equal(b[key].astype(np.int64), p[key].astype(np.int64), err_msg=key)
    np.testing.assert_array_equal(b["hard"], p["hard"])
    code = codes[0]
    pick = np.nonzero(cidx == 0)[0][:8]
    nn = code.n * code.n
    frames = np.stack([llr[o:o + nn] for o in offs[pick]]).reshape(-1, code.n, code.n)
    r = oracle.decode_product(code, frames, 4, 3000, 4, nthreads=8)
    np.testing.assert_array_equal(b["sum_queries"][pick].astype(np.int64), r["sum_queries"].astype(np.int64))
    np.testing.assert_array_equal(b["half_iters"][pick].astype(np.int64), r["half_iters"].astype(np.int64))


def test_batched_matches_oracle_on_sample(sg):
    codes, cidx, eb, offs, llr, cw = mixed(240, seed=7, lo=2.5, hi=3.5)
    b = run_batched(sg, codes, cidx, offs, llr, qcap=3000, iters=4)
    rng = np.random.default_rng(3)
    for c, code in enumerate(codes):
        sel = np.nonzero(cidx == c)[0]
        pick = rng.choice(sel, size=min(6, sel.size), replace=False)
        nn = code.n * code.n
        frames = np.stack([llr[o:o + nn] for o in offs[pick]]).reshape(-1, code.n, code.n)
        r = oracle.decode_product(code, frames, 4, 3000, 4, nthreads=8)
        for j, f in enumerate(pick):
            o = offs[f]
            assert b["success"][f] == r["success"][j]
            assert int(b["half_iters"][f]) == int(r["half_iters"][j])
            assert int(b["sum_queries"][f]) == int(r["sum_queries"][j])
            assert int(b["sum_max_queries"][f]) == int(r["sum_max_queries"][j])
            np.testing.assert_array_equal(b["hard"][o:o + nn], r["hard"][j].reshape(-1))


def test_batched_result_independent_of_launch_shape(sg):
    codes, cidx, eb, offs, llr, cw = mixed(300, seed=9)
    ref = None
    # hand-picked shapes, then every value the library's tuner tries (waves 4/8/16, frames 1-4,
    # chunks 1/2/4/8) at as many groups per compute unit as fit
    for w, fpg, ch, gpc in [(8, 4, 1, 2), (4, 1, 1, 1), (16, 8, 3, 1), (4, 2, 64, 4), (8, 3, 2, 3),
                            (4, 1, 8, 8), (16, 2, 2, 8), (8, 3, 1, 8), (8, 4, 4, 8)]:
        print(f"[gpu] batched shape w={w} f={fpg} chunk={ch} gpc={gpc}", flush=True)
        out = run_batched(sg, codes, cidx, offs, llr, f32=True, sched=sg.sched(w, fpg, ch, gpc))
        assert int(out["status"][0]) == 0
        if ref is None:
            ref = out
            continue
        for key in ("success", "half_iters", "sum_queries", "sum_max_queries", "hard"):
            np.testing.assert_array_equal(out[key], ref[key], err_msg=key)


def test_batched_skips_invalid_descriptors(sg):
    import torch
    codes, cidx, eb, offs, llr, cw = mixed(40, seed=11)
    cidx = cidx.copy()
    offs = offs.copy()
    cidx[5] = 7                      # no such code
    offs[9] = llr.shape[0] - 10      # block runs past the buffer
    out = run_batched(sg, codes, cidx, offs, llr, f32=True, qcap=1000, iters=2)
    assert int(out["status"][0]) & 2
    assert out["success"][5] == 0 and out["half_iters"][5] == 0
    assert out["success"][9] == 0 and out["half_iters"][9] == 0
    good = np.ones(40, bool)
    good[[5, 9]] = False
    assert np.all(out["half_iters"][good] >= 1)


def test_batched_single_frame_and_empty(sg):
    codes, cidx, eb, offs, llr, cw = mixed(1, seed=12)
    b = run_batched(sg, codes, cidx, offs, llr)
    p = run_plain_per_code(sg, codes, cidx, offs, llr)
    np.testing.assert_array_equal(b["hard"], p["hard"])


def test_tuned_shape_gives_identical_results(sg):
    """The library's tuner picks a shape on a sample and records it; decoding with that shape, and
    with no shape (the recorded one), gives the default shape's per-frame results."""
    import torch
    codes, cidx, eb, offs, llr, cw = mixed(200, seed=21)
    gcodes = [handle(sg, c) for c in codes]
    x = torch.from_numpy(llr.astype(np.float32)).cuda()
    fc, fo = torch.from_numpy(cidx).cuda(), torch.from_numpy(offs).cuda()
    sg.sched_table_clear()
    print("[gpu] tuner on 200 mixed frames", flush=True)
    best, ms = sg.sched_tune(gcodes, fc, fo, x, list_max=4, query_cap=3000, max_iter=4)
    assert ms > 0.0
    assert best.waves_per_group in (4, 8, 16) and 1 <= best.frames_per_group <= 4
    assert best.steal_chunk in (1, 2, 4, 8) and best.groups_per_cu == sg.sched().groups_per_cu
    ref = run_batched(sg, codes, cidx, offs, llr, f32=True, sched=sg.sched(), qcap=3000, iters=4)
    tuned = run_batched(sg, codes, cidx, offs, llr, f32=True, sched=best, qcap=3000, iters=4)
    recorded = run_batched(sg, codes, cidx, offs, llr, f32=True, sched=None, qcap=3000, iters=4)
    sg.sched_table_clear()
    for out in (tuned, recorded):
        assert int(out["status"][0]) == 0
        for key in ("success", "half_iters", "sum_queries", "sum_max_queries", "hard"):
            np.testing.assert_array_equal(out[key], ref[key], err_msg=key)


@pytest.mark.parametrize("last_present", [True, False])
def test_batched_frame_order_cases(sg, last_present):
    """Frames are taken in an order of the library's choosing (longest code first, the shortest
    code's frames by their mean |L|): with more frames than one pass of the order kernel covers,
    two codes of equal length (the later one is taken last), and invalid descriptors among them,
    every valid frame still gets the plain path's result.  Without last_present, the code taken
    last has no frames in the batch."""
    nks = [(64, 57), (32, 26), (32, 26)]
    codes, cidx, eb, offs, llr, cw = mixed(3000, seed=31, nks=nks)
    cidx = cidx.copy()
    offs = offs.copy()
    if not last_present:
        cidx[cidx == 2] = 1          # same length, so the blocks stay where they are
    bad = np.array([3, 1500, 2999])
    cidx[bad[0]] = 9                 # no such code
    offs[bad[1]] = llr.shape[0] - 5  # block runs past the buffer
    cidx[bad[2]] = 200
    print(f"[gpu] batched order cases, last code present={last_present}", flush=True)
    b = run_batched(sg, codes, cidx, offs, llr, f32=True, qcap=1000, iters=2)
    assert int(b["status"][0]) & 2
    good = np.ones(cidx.shape[0], bool)
    good[bad] = False
    assert np.all(b["success"][bad] == 0) and np.all(b["half_iters"][bad] == 0)
    p = run_plain_per_code(sg, codes, np.where(good, cidx, 255), offs, llr, f32=True, qcap=1000, iters=2)
    for key in ("success", "half_iters", "sum_queries", "sum_max_queries"):
        np.testing.assert_array_equal(b[key][good], p[key][good], err_msg=key)
    for f in np.nonzero(good)[0]:
        nn = codes[cidx[f]].n ** 2
        np.testing.assert_array_equal(b["hard"][offs[f]:offs[f] + nn], p["hard"][offs[f]:offs[f] + nn])
