"""Serving (continuous batching of product-frame requests): every served result equals the
plain path's decode of the same frame alone, whatever else is in flight; admission by device
memory refuses and then recovers; poll semantics; timestamps; parity with the oracle on a
sample."""
import ctypes
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


def frames_of(F, seed, lo=2.5, hi=4.0, nks=NK):
    codes = [synth.ebch(*nk) for nk in nks]
    cidx, eb, offs, llr, cw = synth.mixed_product_frames(codes, lo, hi, seed, np.arange(F))
    out = []
    for f in range(F):
        c = codes[cidx[f]]
        out.append((int(cidx[f]), llr[offs[f]:offs[f] + c.n * c.n].reshape(c.n, c.n)))
    return codes, out


def alone(sg, code, gcode, llr, f32, L, qcap, iters, early_stop=True):
    """Plain-path decode of each frame by itself (one call per frame)."""
    import torch
    dt = torch.float32 if f32 else torch.float64
    res = []
    for x in llr:
        o = sg.sogrand_decode_product(gcode, torch.from_numpy(np.ascontiguousarray(x)).to(dtype=dt, device="cuda")
                                      .reshape(1, code.n, code.n), list_max=L, query_cap=qcap, max_iter=iters,
                                      early_stop=early_stop)
        torch.cuda.synchronize()
        res.append(dict(hard=o["hard"][0].cpu().numpy(), success=int(o["success"][0]),
                        half_iters=int(o["half_iters"][0]), queries=int(o["sum_queries"][0])))
    return res


def serve_all(sg, srv, gcodes, frames, f32, batch=40):
    """Submits in waves, polling between waves so that new frames join frames in flight."""
    dt = np.float32 if f32 else np.float64
    results, ids = {}, {}
    pend = list(range(len(frames)))
    while pend or len(results) < len(frames):
        k = 0
        while pend and k < batch:
            f = pend[0]
            ci, x = frames[f]
            rid = srv.submit(gcodes[ci], np.ascontiguousarray(x, dtype=dt), tag=f)
            if rid is None:
                break
            ids[rid] = f
            pend.pop(0)
            k += 1
        for r in srv.poll(max_results=64, timeout_ns=2_000_000):
            assert ids[r["request_id"]] == r["user_tag"]
            results[r["user_tag"]] = r
    return results


@pytest.mark.parametrize("f32", [True, False])
def test_served_results_equal_alone(sg, f32):
    F, L, qcap, iters = 90, 4, 2000, 4
    codes, frames = frames_of(F, seed=6)
    print(f"[gpu] serve {F} mixed frames f32={f32}", flush=True)
    gcodes = [sg.Code.ebch(c.n, c.k) for c in codes]
    prec = sg.SOGRAND_F32 if f32 else sg.SOGRAND_F64
    with sg.Server(64 << 20, list_max=L, query_cap=qcap, max_iter=iters, precision=prec) as srv:
        got = serve_all(sg, srv, gcodes, frames, f32)
        st = srv.stats()
    assert len(got) == F and st["frames"] == F and st["steps"] >= 1
    for ci, code in enumerate(codes):
        sel = [f for f in range(F) if frames[f][0] == ci]
        ref = alone(sg, code, gcodes[ci], [frames[f][1] for f in sel], f32, L, qcap, iters)
        for f, r in zip(sel, ref):
            g = got[f]
            assert g["status"] == 0 and g["n"] == code.n
            assert (g["success"], g["half_iters"], g["queries"]) == (r["success"], r["half_iters"], r["queries"]), f
            np.testing.assert_array_equal(g["hard"], r["hard"], err_msg=f"frame {f}")
            assert g["t_submit_ns"] <= g["t_admit_ns"] <= g["t_done_ns"]


def test_served_short_and_odd_codes(sg):
    """Requests of the non-even odd-length Hamming[15,11], of [8,4] and of [64,57] in one server:
    each result equals the frame decoded alone."""
    base = synth.ebch(16, 11)
    codes = [synth.code_from_generator("Hamming[15,11]", base.G[:, :15], base.info_pos), synth.ebch(8, 4),
             synth.ebch(64, 57)]
    F, L, qcap, iters = 60, 4, 2000, 4
    cidx, eb, offs, llr, cw = synth.mixed_product_frames(codes, 2.0, 3.5, 17, np.arange(F))
    frames = [(int(cidx[f]), llr[offs[f]:offs[f] + codes[cidx[f]].n ** 2].reshape(codes[cidx[f]].n, -1))
              for f in range(F)]
    print(f"[gpu] serve {F} frames of Hamming[15,11], [8,4], [64,57]", flush=True)
    gcodes = [sg.Code.from_hcols(c.n, c.k, c.hcols) for c in codes]
    with sg.Server(64 << 20, list_max=L, query_cap=qcap, max_iter=iters, precision=sg.SOGRAND_F32) as srv:
        got = serve_all(sg, srv, gcodes, frames, True)
    assert len(got) == F
    for ci, code in enumerate(codes):
        sel = [f for f in range(F) if frames[f][0] == ci]
        ref = alone(sg, code, gcodes[ci], [frames[f][1] for f in sel], True, L, qcap, iters)
        for f, r in zip(sel, ref):
            g = got[f]
            assert g["status"] == 0 and g["n"] == code.n
            assert (g["success"], g["half_iters"], g["queries"]) == (r["success"], r["half_iters"], r["queries"]), f
            np.testing.assert_array_equal(g["hard"], r["hard"], err_msg=f"frame {f}")


def test_served_matches_oracle_sample(sg):
    F, L, qcap, iters = 24, 4, 1000, 4
    code = synth.ebch(32, 26)
    llr, cw, _ = synth.product_frames(code, 3.0, 0, np.arange(F))
    llr32 = llr.astype(np.float32)
    g = sg.Code.ebch(32, 26)
    with sg.Server(8 << 20, list_max=L, query_cap=qcap, max_iter=iters, precision=sg.SOGRAND_F32) as srv:
        got = serve_all(sg, srv, [g], [(0, llr32[f]) for f in range(F)], True)
    ref = oracle.decode_product(code, llr32.astype(np.float64), L, qcap, iters, store_f32=True)
    for f in range(F):
        assert got[f]["success"] == int(ref["success"][f])
        assert got[f]["half_iters"] == int(ref["half_iters"][f])
        assert got[f]["queries"] == int(ref["sum_queries"][f])
        np.testing.assert_array_equal(got[f]["hard"], ref["hard"][f])


def test_admission_by_memory(sg):
    """A 1 MiB pool holds seven FP32 [128,120]^2 slots: a further submission is refused until
    results are taken; refused frames are admitted as slots free and decoded like the others.  Without
    early stopping every frame runs all six half-iterations, so the pool is still full when the
    eighth frame arrives."""
    code = synth.ebch(128, 120)
    g = sg.Code.ebch(128, 120)
    llr, _, _ = synth.product_frames(code, 3.5, 7, np.arange(10))
    x = llr.astype(np.float32)
    with sg.Server(1 << 20, list_max=4, query_cap=1000, max_iter=3, early_stop=False,
                   precision=sg.SOGRAND_F32) as srv:
        ids = []
        for f in range(10):
            rid = srv.submit(g, np.ascontiguousarray(x[f]), tag=f)
            if rid is None:
                break
            ids.append(rid)
        admitted = len(ids)
        assert 1 <= admitted < 10
        got = {}
        while len(got) < admitted:
            for r in srv.poll(max_results=16, timeout_ns=-1):
                got[r["user_tag"]] = r
        # the rest: each refusal is followed by a poll that frees a slot
        pending = list(range(admitted, 10))
        while pending or len(got) < 10:
            if pending and srv.submit(g, np.ascontiguousarray(x[pending[0]]), tag=pending[0]) is not None:
                pending.pop(0)
                continue
            for r in srv.poll(max_results=16, timeout_ns=-1):
                got[r["user_tag"]] = r
    ref = alone(sg, code, g, list(x), True, 4, 1000, 3, early_stop=False)
    for f in range(10):
        np.testing.assert_array_equal(got[f]["hard"], ref[f]["hard"])
        assert got[f]["half_iters"] == ref[f]["half_iters"]


def test_poll_semantics(sg):
    L = sg.lib()
    code = synth.ebch(32, 26)
    g = sg.Code.ebch(32, 26)
    llr, _, _ = synth.product_frames(code, 4.0, 8, np.arange(1))
    srv = sg.Server(4 << 20, list_max=4, query_cap=1000, max_iter=4, precision=sg.SOGRAND_F64)
    try:
        res = (sg.sogrand_result_t * 4)()
        n = ctypes.c_size_t()
        # nothing in flight
        assert L.sogrand_serve_poll(srv._h, res, 4, ctypes.byref(n), None, None, 0) == sg.SOGRAND_ENOTFOUND
        assert L.sogrand_serve_poll(srv._h, res, 4, ctypes.byref(n), None, None, -1) == sg.SOGRAND_ENOTFOUND
        assert srv.submit(g, np.ascontiguousarray(llr[0])) is not None
        rc = L.sogrand_serve_poll(srv._h, res, 4, ctypes.byref(n), None, None, -1)
        assert rc == 0 and n.value == 1 and res[0].status == 0
        # taken: nothing left
        assert L.sogrand_serve_poll(srv._h, res, 4, ctypes.byref(n), None, None, 1000) == sg.SOGRAND_ENOTFOUND
        # wrong dtype or size is refused by the binding; a NULL LLR pointer by the library
        with pytest.raises(ValueError):
            srv.submit(g, np.zeros((32, 32), np.float32))
        rid = ctypes.c_uint64()
        assert L.sogrand_serve_submit(srv._h, g.handle, None, 0, ctypes.byref(rid)) == -1
    finally:
        srv.close()


def test_destroy_finishes_admitted_work(sg):
    code = synth.ebch(64, 57)
    g = sg.Code.ebch(64, 57)
    llr, _, _ = synth.product_frames(code, 3.0, 9, np.arange(20))
    srv = sg.Server(16 << 20, list_max=4, query_cap=1000, max_iter=4, precision=sg.SOGRAND_F32)
    for f in range(20):
        assert srv.submit(g, np.ascontiguousarray(llr[f].astype(np.float32)), tag=f) is not None
    srv.close()   # returns once every admitted frame has been decoded
