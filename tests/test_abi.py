"""Host-side checks of the C ABI: the library loads, exports every declared
function, builds the same codes as the input generator, and rejects bad
arguments before touching a GPU.  No decoding call runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sg():
    import paper_2310_10737_amd as sg
    # the sanitizer test runs this module against a host-only build of the library
    other = os.environ.get("SOGRAND_TEST_LIBRARY")
    if other:
        sg._LIBPATH = other
    elif not os.path.exists(sg.library_path()):
        from paper_2310_10737_amd import build
        build.build()
    sg.lib()
    return sg


def declared_functions():
    names = []
    for path in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not path.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", path)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(sogrand_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(sg):
    names = declared_functions()
    assert "sogrand_decode_component" in names and "sogrand_decode_product" in names
    L = ctypes.CDLL(sg.library_path())
    for name in names:
        assert hasattr(L, name), name
    assert set(sg.EXPORTS) <= set(names)


def test_version_and_defaults(sg):
    assert sg.lib().sogrand_version() >= 100
    p = sg.sogrand_params_t()
    sg.lib().sogrand_params_default(ctypes.byref(p))
    assert (p.list_max, p.query_cap, p.alpha, p.max_iter, p.early_stop, p.precision) == (4, 1000, 0.5, 4, 1, 0)
    assert p.list_bler_stop == 0.0
    assert ctypes.sizeof(sg.sogrand_params_t) == 40   # the C layout


@pytest.mark.parametrize("nk", [(8, 4), (16, 11), (32, 26), (64, 57), (128, 120), (16, 7)])
def test_library_ebch_is_the_same_code(sg, nk):
    code = sg.Code.ebch(*nk)
    ref = synth.ebch(*nk)
    assert (code.n, code.k, code.is_even) == (ref.n, ref.k, True)
    h = np.array(code.hcols(), dtype=np.uint64)
    H = ((h[None, :] >> np.arange(code.n - code.k, dtype=np.uint64)[:, None]) & np.uint64(1)).astype(np.int64)
    # every codeword of the generator's code passes the library's checks, and H has full rank
    assert not np.any((ref.G.astype(np.int64) @ H.T) % 2)
    assert np.linalg.matrix_rank(H.astype(float)) == code.n - code.k


def test_code_create_from_columns_and_evenness(sg):
    ref = synth.ebch(16, 11)
    c = sg.Code.from_hcols(16, 11, ref.hcols)
    assert c.is_even and c.hcols() == list(ref.hcols)
    base = synth.ebch(16, 11)
    ham = synth.code_from_generator("h15", base.G[:, :15], base.info_pos)
    c2 = sg.Code.from_hcols(15, 11, ham.hcols)
    assert not c2.is_even


@pytest.mark.parametrize("n,k,cols", [
    (16, 11, [1] * 16),                  # rank 1
    (200, 190, [1] * 200),               # n too large
    (16, 11, [1 << 6] + [1] * 15),       # bit above row n-k-1
])
def test_code_create_rejects_bad_h(sg, n, k, cols):
    with pytest.raises(sg.SograndError) as e:
        sg.Code.from_hcols(n, k, cols)
    assert e.value.code == -1


def test_ebch_rejects_unknown_parameters(sg):
    with pytest.raises(sg.SograndError):
        sg.Code.ebch(32, 20)
    with pytest.raises(sg.SograndError):
        sg.Code.ebch(256, 247)


@pytest.mark.parametrize("field,value", [
    ("list_max", 0), ("list_max", 17), ("query_cap", 0), ("query_cap", (1 << 24) + 1),
    ("alpha", 0.0), ("alpha", float("nan")), ("max_iter", 0), ("precision", 2),
    ("list_bler_stop", -0.1), ("list_bler_stop", 1.5), ("list_bler_stop", float("nan")),
])
def test_decode_rejects_bad_params_before_device_work(sg, field, value):
    code = sg.Code.ebch(32, 26)
    p = sg.params()
    setattr(p, field, value)
    L = sg.lib()
    rc = L.sogrand_decode_component(code.handle, ctypes.byref(p), 1, ctypes.c_void_p(1), *([None] * 9), None)
    assert rc == -1 and L.sogrand_last_error()
    rc = L.sogrand_decode_product(code.handle, ctypes.byref(p), 1, ctypes.c_void_p(1), ctypes.c_void_p(1), None,
                                  ctypes.c_void_p(1), None, None, None, None)
    assert rc == -1


def test_decode_rejects_null_buffers_and_accepts_empty_batches(sg):
    code = sg.Code.ebch(32, 26)
    p = sg.params()
    L = sg.lib()
    assert L.sogrand_decode_component(code.handle, ctypes.byref(p), 0, None, *([None] * 9), None) == 0
    assert L.sogrand_decode_component(code.handle, ctypes.byref(p), 5, None, *([None] * 9), None) == -1
    assert L.sogrand_decode_product(code.handle, ctypes.byref(p), 0, None, None, None, None, None, None, None, None) == 0
    assert L.sogrand_decode_product(code.handle, ctypes.byref(p), 3, ctypes.c_void_p(1), None, None,
                                    ctypes.c_void_p(1), None, None, None, None) == -1
    assert L.sogrand_decode_component(None, ctypes.byref(p), 1, ctypes.c_void_p(1), *([None] * 9), None) == -1


def test_batched_rejects_bad_arguments_before_device_work(sg):
    code = sg.Code.ebch(32, 26)
    L = sg.lib()
    p = sg.params()
    one = (ctypes.c_void_p * 1)(code.handle)
    sc = sg.sched()
    args = [one, 1, ctypes.byref(p), 4, ctypes.c_void_p(1), ctypes.c_void_p(1), 4096, ctypes.c_void_p(1),
            ctypes.c_void_p(1), None, ctypes.c_void_p(1), None, None, None, None, ctypes.byref(sc), None]
    bad_ncodes = list(args)
    bad_ncodes[1] = 0
    assert L.sogrand_decode_batched(*bad_ncodes) == -1
    bad_ncodes[1] = 9
    assert L.sogrand_decode_batched(*bad_ncodes) == -1
    no_success = list(args)
    no_success[10] = None
    assert L.sogrand_decode_batched(*no_success) == -1
    for field, value in (("waves_per_group", 5), ("frames_per_group", 0), ("frames_per_group", 9),
                         ("steal_chunk", 0), ("groups_per_cu", 0)):
        bad = sg.sched()
        setattr(bad, field, value)
        a = list(args)
        a[15] = ctypes.byref(bad)
        assert L.sogrand_decode_batched(*a) == -1, field
    empty = list(args)
    empty[3] = 0
    assert L.sogrand_decode_batched(*empty) == 0


def test_serving_rejects_bad_arguments_before_device_work(sg):
    L = sg.lib()
    p = sg.params()
    out = ctypes.c_void_p()
    assert L.sogrand_serve_create(ctypes.byref(p), 1 << 10, 0, ctypes.byref(out)) == -1   # budget below 1 MiB
    assert L.sogrand_serve_create(ctypes.byref(p), 1 << 30, 0, None) == -1
    assert L.sogrand_serve_create(ctypes.byref(p), 1 << 30, 2, ctypes.byref(out)) == -1   # unknown flag
    bad = sg.params()
    bad.list_max = 0
    assert L.sogrand_serve_create(ctypes.byref(bad), 1 << 30, 0, ctypes.byref(out)) == -1
    assert not out.value
    rid = ctypes.c_uint64()
    code = sg.Code.ebch(32, 26)
    assert L.sogrand_serve_submit(None, code.handle, ctypes.c_void_p(1), 0, ctypes.byref(rid)) == -1
    res = (sg.sogrand_result_t * 2)()
    n = ctypes.c_size_t()
    assert L.sogrand_serve_poll(None, res, 2, ctypes.byref(n), None, None, 0) == -1
    assert L.sogrand_serve_stats(None, None) == -1
    assert L.sogrand_serve_destroy(None) == 0
    assert L.sogrand_clock_ns() > 0
    assert ctypes.sizeof(sg.sogrand_result_t) == 72   # the C layout (natural alignment)


def test_tuned_shape_table_round_trip(sg, tmp_path):
    """The table of tuned launch shapes is host state: a saved file loads back entry for entry,
    and a malformed or out-of-range line is refused without adding anything."""
    sg.sched_table_clear()
    good = tmp_path / "tuned.txt"
    good.write_text("product f32 nostop 32:26 64:57 128:120|8 2 4 8\n"
                    "gldpc f64 stop 32:26|16 3 1 2\n")
    assert sg.sched_table_load(str(good)) == 2
    saved = tmp_path / "saved.txt"
    sg.sched_table_save(str(saved))
    assert sorted(saved.read_text().splitlines()) == sorted(good.read_text().splitlines())
    for bad in ("product f32 nostop 64:57|8 2 4\n",          # a field missing
                "product f32 nostop 64:57|5 2 4 8\n",        # waves_per_group not 4, 8 or 16
                "product f32 nostop 64:57|8 2 4 8 9\n",      # a field too many
                "|8 2 4 8\n",                                # no kind
                "product f32 nostop 64:57 8 2 4 8\n"):       # no separator
        p = tmp_path / "bad.txt"
        p.write_text("product f64 nostop 8:4|4 1 1 1\n" + bad)
        with pytest.raises(sg.SograndError):
            sg.sched_table_load(str(p))
    sg.sched_table_save(str(saved))
    assert len(saved.read_text().splitlines()) == 2     # nothing from the refused files
    with pytest.raises(sg.SograndError):
        sg.sched_table_load(str(tmp_path / "missing.txt"))
    sg.sched_table_clear()
    sg.sched_table_save(str(saved))
    assert saved.read_text() == ""


def test_plan_rejects_bad_arguments_before_device_work(sg):
    L = sg.lib()
    p = sg.params()
    one = ctypes.c_void_p(1)
    out = ctypes.c_void_p()
    code = sg.Code.ebch(8, 4)
    ok = [code.handle, ctypes.byref(p), 4, 0, one, one, None, one, None, None, None, ctypes.byref(out)]
    for i, value in ((0, None), (2, 0), (4, None), (5, None), (7, None), (11, None)):
        a = list(ok)
        a[i] = value
        assert L.sogrand_plan_create(*a) == -1, i
    assert L.sogrand_plan_launch(None, None) == -1
    L.sogrand_plan_destroy(None)
