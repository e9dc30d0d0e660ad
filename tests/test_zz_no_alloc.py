"""The product decode entry point that allocates nothing (sogrand_decode_product_noalloc): the
same results as sogrand_decode_product, called through the C ABI, twice in a row with the second
call smaller than the first (the static work buffer keeps the first call's contents, which must
not leak into the second); and its refusals, which touch no device memory."""
import ctypes
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    sg.lib()
    return sg


def run(sg, fn, code, x, **kw):
    import torch
    out = fn(code, x, want_app=True, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


@pytest.mark.parametrize("nk,ebn0,sizes,f32", [((64, 57), 2.75, (300, 77), True), ((32, 26), 2.5, (500, 3), False),
                                               ((128, 120), 3.0, (40, 9), True)])
def test_noalloc_equals_allocating_path_twice(sg, nk, ebn0, sizes, f32):
    import torch
    code = synth.ebch(*nk)
    g = sg.Code.ebch(*nk)
    dt = torch.float32 if f32 else torch.float64
    kw = dict(list_max=4, query_cap=3000, max_iter=4)
    for call, F in enumerate(sizes):
        llr, _, _ = synth.product_frames(code, ebn0, 200 + call, np.arange(F))
        x = torch.from_numpy(llr).to(dtype=dt, device="cuda")
        print(f"[gpu] noalloc {code.name}^2 call {call}: {F} frames f32={f32}", flush=True)
        want = run(sg, sg.sogrand_decode_product, g, x, **kw)       # also builds the code's tables
        got = run(sg, sg.sogrand_decode_product_noalloc, g, x, **kw)
        for key in ("hard", "success", "half_iters", "sum_queries", "sum_max_queries", "llr_app"):
            np.testing.assert_array_equal(got[key], want[key], err_msg=f"call {call}: {key}")
        assert want["half_iters"].max() > 1


def test_noalloc_refuses_without_device_work(sg):
    import torch
    L = sg.lib()
    code = sg.Code.ebch(64, 57)
    x = torch.zeros((4, 64, 64), dtype=torch.float32, device="cuda")
    # a fresh handle has no device tables yet, and this call may not build them
    with pytest.raises(sg.SograndError) as e:
        sg.sogrand_decode_product_noalloc(code, x, query_cap=500)
    assert e.value.code == -1 and "not built" in str(e.value)
    # more frames than the static buffer holds: refused before any table is looked at
    p = sg.params(precision=sg.SOGRAND_F64)
    big = sg.SOGRAND_NOALLOC_WORK_MAX // (3 * 64 * 64 * 8) + 1
    rc = L.sogrand_decode_product_noalloc(code.handle, ctypes.byref(p), big, ctypes.c_void_p(1),
                                          ctypes.c_void_p(1), None, ctypes.c_void_p(1), None, None, None, None)
    assert rc == -1 and b"static buffer" in L.sogrand_last_error()
    assert L.sogrand_decode_product_noalloc(code.handle, ctypes.byref(p), 0, None, None, None, None, None, None,
                                            None, None) == 0
