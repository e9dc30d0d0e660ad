"""Python binding of libsogrand (SOGRAND decoding of product codes on MI355X).

Argument marshalling only: every decoding step runs in the HIP kernels of
``libsogrand.so`` behind the C ABI declared in ``include/sogrand.h``.  PyTorch
provides device memory and the current HIP stream.  There is no fallback: if
the shared library is missing, every call raises ``SograndError``.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "SograndError", "Code", "params", "sched", "lib", "library_path", "profile_begin", "profile_end",
    "sogrand_decode_component", "sogrand_decode_product", "sogrand_decode_product_noalloc", "sogrand_decode_gldpc",
    "sogrand_decode_batched", "sogrand_decode_batched_gldpc", "pack_frames",
    "Server", "sogrand_clock_ns", "measure_valu_rate", "SOGRAND_F64", "SOGRAND_F32",
]

SOGRAND_F64 = 0
SOGRAND_F32 = 1
SOGRAND_NOALLOC_WORK_MAX = 64 << 20
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libsogrand.so")
_lib = None

EXPORTS = [
    "sogrand_last_error", "sogrand_version", "sogrand_params_default",
    "sogrand_code_create", "sogrand_code_create_ebch", "sogrand_code_info", "sogrand_code_destroy",
    "sogrand_decode_component", "sogrand_decode_product", "sogrand_decode_product_noalloc", "sogrand_decode_gldpc",
    "sogrand_sched_default", "sogrand_decode_batched", "sogrand_decode_batched_gldpc",
    "sogrand_sched_tune", "sogrand_sched_table_save", "sogrand_sched_table_load", "sogrand_sched_table_clear",
    "sogrand_plan_create", "sogrand_plan_launch", "sogrand_plan_destroy",
    "sogrand_clock_ns", "sogrand_serve_create", "sogrand_serve_submit", "sogrand_serve_poll",
    "sogrand_serve_stats", "sogrand_serve_replay", "sogrand_serve_destroy",
    "sogrand_profile_begin", "sogrand_profile_end", "sogrand_measure_valu_rate",
]

SOGRAND_SERVE_APP = 1
SOGRAND_EAGAIN = -4
SOGRAND_ENOTFOUND = -5
SOGRAND_ETIMEDOUT = -6


class SograndError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsogrand error {code}: {msg}")
        self.code = code


class sogrand_kernel_stat_t(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_char * 48),
        ("launches", ctypes.c_uint64),
        ("total_ms", ctypes.c_double),
        ("words", ctypes.c_uint64),
        ("queries", ctypes.c_uint64),
        ("ranks", ctypes.c_uint64),
        ("exact_rank", ctypes.c_uint64),
        ("phase_cycles", ctypes.c_uint64 * 8),
    ]


class sogrand_sched_t(ctypes.Structure):
    _fields_ = [
        ("waves_per_group", ctypes.c_int),
        ("frames_per_group", ctypes.c_int),
        ("steal_chunk", ctypes.c_int),
        ("groups_per_cu", ctypes.c_int),
    ]


class sogrand_result_t(ctypes.Structure):
    _fields_ = [
        ("request_id", ctypes.c_uint64),
        ("user_tag", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("success", ctypes.c_uint8),
        ("half_iters", ctypes.c_uint16),
        ("n", ctypes.c_uint16),
        ("queries", ctypes.c_uint64),
        ("hard_offset", ctypes.c_uint64),
        ("t_submit_ns", ctypes.c_uint64),
        ("t_admit_ns", ctypes.c_uint64),
        ("t_done_ns", ctypes.c_uint64),
    ]


class sogrand_serve_stats_t(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_uint64),
        ("frames", ctypes.c_uint64),
        ("max_active", ctypes.c_uint64),
        ("step_ms", ctypes.c_double),
        ("max_step_ms", ctypes.c_double),
        ("host_ms", ctypes.c_double),
    ]


class sogrand_params_t(ctypes.Structure):
    _fields_ = [
        ("list_max", ctypes.c_int),
        ("query_cap", ctypes.c_uint32),
        ("alpha", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("early_stop", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("list_bler_stop", ctypes.c_double),
    ]


def library_path() -> str:
    return _LIBPATH


def lib():
    """The loaded libsogrand (raises SograndError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        raise SograndError(-3, f"{_LIBPATH} is missing: build it with __graft_entry__.build()")
    # torch (which supplies device memory and streams) loads its HIP runtime first, so that the
    # library binds to the same runtime instead of loading a second one into the process
    import torch  # noqa: F401
    L = ctypes.CDLL(_LIBPATH)
    P, I, U32, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_size_t
    L.sogrand_last_error.restype = ctypes.c_char_p
    L.sogrand_version.restype = I
    L.sogrand_params_default.argtypes = [P]
    L.sogrand_code_create.argtypes = [I, I, P, P]
    L.sogrand_code_create_ebch.argtypes = [I, I, P]
    L.sogrand_code_info.argtypes = [P, P, P, P, P]
    L.sogrand_code_destroy.argtypes = [P]
    L.sogrand_code_destroy.restype = None
    L.sogrand_decode_component.argtypes = [P, P, SZ] + [P] * 11
    L.sogrand_decode_product.argtypes = [P, P, SZ] + [P] * 8
    L.sogrand_decode_product_noalloc.argtypes = [P, P, SZ] + [P] * 8
    L.sogrand_decode_gldpc.argtypes = [P, P, SZ] + [P] * 8
    L.sogrand_sched_default.argtypes = [P]
    L.sogrand_sched_default.restype = None
    L.sogrand_decode_batched.argtypes = [P, I, P, SZ, P, P, ctypes.c_uint64] + [P] * 10
    L.sogrand_decode_batched_gldpc.argtypes = [P, I, P, SZ, P, P, ctypes.c_uint64] + [P] * 10
    L.sogrand_plan_create.argtypes = [P, P, SZ, I] + [P] * 8
    L.sogrand_plan_launch.argtypes = [P, P]
    L.sogrand_plan_destroy.argtypes = [P]
    L.sogrand_plan_destroy.restype = None
    L.sogrand_sched_tune.argtypes = [I, P, I, P, SZ, P, P, ctypes.c_uint64, P, P, P, P]
    L.sogrand_sched_table_save.argtypes = [ctypes.c_char_p]
    L.sogrand_sched_table_load.argtypes = [ctypes.c_char_p]
    L.sogrand_sched_table_clear.restype = None
    L.sogrand_clock_ns.restype = ctypes.c_uint64
    L.sogrand_serve_create.argtypes = [P, SZ, ctypes.c_uint, P]
    L.sogrand_serve_submit.argtypes = [P, P, P, ctypes.c_uint64, P]
    L.sogrand_serve_poll.argtypes = [P, P, SZ, P, P, P, ctypes.c_int64]
    L.sogrand_serve_stats.argtypes = [P, P]
    L.sogrand_serve_replay.argtypes = [P, P, I, SZ, P, P, P, ctypes.c_uint64, P, ctypes.c_uint64, P]
    L.sogrand_serve_destroy.argtypes = [P]
    L.sogrand_profile_begin.argtypes = [I]
    L.sogrand_profile_end.argtypes = [P, I, P]
    L.sogrand_measure_valu_rate.argtypes = [I, P, P, P]
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise SograndError(rc, lib().sogrand_last_error().decode())


class Code:
    """A binary linear [n, k] code handle (library-owned, immutable)."""

    def __init__(self, handle, n, k, even):
        self._h = handle
        self.n, self.k, self.is_even = n, k, bool(even)

    @classmethod
    def ebch(cls, n: int, k: int) -> "Code":
        h = ctypes.c_void_p()
        _check(lib().sogrand_code_create_ebch(n, k, ctypes.byref(h)))
        return cls._wrap(h)

    @classmethod
    def from_hcols(cls, n: int, k: int, hcols) -> "Code":
        arr = (ctypes.c_uint32 * n)(*[int(x) for x in hcols])
        h = ctypes.c_void_p()
        _check(lib().sogrand_code_create(n, k, arr, ctypes.byref(h)))
        return cls._wrap(h)

    @classmethod
    def _wrap(cls, h):
        n, k, ev = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().sogrand_code_info(h, ctypes.byref(n), ctypes.byref(k), ctypes.byref(ev), None))
        return cls(h, n.value, k.value, ev.value)

    def hcols(self):
        arr = (ctypes.c_uint32 * self.n)()
        _check(lib().sogrand_code_info(self._h, None, None, None, arr))
        return [int(x) for x in arr]

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.sogrand_code_destroy(self._h)
            self._h = None


def profile_begin(count_work: bool = False):
    """Bracket every decode kernel launched from now on with HIP events (and count work)."""
    _check(lib().sogrand_profile_begin(int(bool(count_work))))


def profile_end():
    """Per-kernel-family totals since profile_begin: {name: dict(launches, total_ms, words, queries, ranks)}."""
    arr = (sogrand_kernel_stat_t * 16)()
    n = ctypes.c_int()
    _check(lib().sogrand_profile_end(arr, 16, ctypes.byref(n)))
    return {arr[i].kernel.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms, words=arr[i].words,
                                         queries=arr[i].queries, ranks=arr[i].ranks,
                                         exact_rank=arr[i].exact_rank,
                                         phase_cycles=[int(x) for x in arr[i].phase_cycles])
            for i in range(n.value)}


def params(list_max=4, query_cap=1000, alpha=0.5, max_iter=4, early_stop=True, precision=SOGRAND_F64,
           list_bler_stop=0.0):
    p = sogrand_params_t()
    p.list_max, p.query_cap, p.alpha = int(list_max), int(query_cap), float(alpha)
    p.max_iter, p.early_stop, p.precision = int(max_iter), int(bool(early_stop)), int(precision)
    p.list_bler_stop = float(list_bler_stop)
    return p


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _precision_of(t):
    import torch
    if t.dtype == torch.float64:
        return SOGRAND_F64
    if t.dtype == torch.float32:
        return SOGRAND_F32
    raise TypeError("LLR tensors must be float64 or float32")


def sogrand_decode_component(code: Code, llr_in, list_max=4, query_cap=1000, found_z=False,
                             outputs=None, stream=None, list_bler_stop=0.0):
    """Component SISO decode of llr_in (W, n) on its device; returns a dict of tensors.

    ``outputs`` may pre-supply any output tensor by name (llr_app, llr_ext, hard,
    n_queries, n_found, found_q, p_found, p_notfound, found_z); a name mapped to
    None is not computed.
    """
    import torch
    if not llr_in.is_cuda or not llr_in.is_contiguous() or llr_in.dim() != 2 or llr_in.shape[1] != code.n:
        raise ValueError("llr_in must be a contiguous CUDA tensor of shape (W, n)")
    W, n = llr_in.shape
    dev, dt = llr_in.device, llr_in.dtype
    L = int(list_max)
    out = dict(
        llr_app=torch.empty((W, n), dtype=dt, device=dev),
        llr_ext=torch.empty((W, n), dtype=dt, device=dev),
        hard=torch.empty((W, n), dtype=torch.uint8, device=dev),
        n_queries=torch.empty(W, dtype=torch.int32, device=dev),
        n_found=torch.empty(W, dtype=torch.uint8, device=dev),
        found_q=torch.empty((W, L), dtype=torch.int32, device=dev),
        p_found=torch.empty((W, L), dtype=torch.float64, device=dev),
        p_notfound=torch.empty(W, dtype=torch.float64, device=dev),
        found_z=torch.empty((W, L, n), dtype=torch.uint8, device=dev) if found_z else None,
    )
    if outputs:
        out.update(outputs)
    p = params(list_max=L, query_cap=query_cap, precision=_precision_of(llr_in), list_bler_stop=list_bler_stop)
    _check(lib().sogrand_decode_component(
        code.handle, ctypes.byref(p), W, _ptr(llr_in), _ptr(out["llr_app"]), _ptr(out["llr_ext"]),
        _ptr(out["hard"]), _ptr(out["n_queries"]), _ptr(out["n_found"]), _ptr(out["found_q"]),
        _ptr(out["p_found"]), _ptr(out["p_notfound"]), _ptr(out["found_z"]), _stream(stream)))
    return out


def sogrand_decode_product(code: Code, llr_ch, list_max=4, query_cap=1000, max_iter=4, alpha=0.5,
                           early_stop=True, want_app=False, outputs=None, stream=None, list_bler_stop=0.0):
    """Block-turbo decode of product-code frames llr_ch (F, n, n); returns a dict of tensors."""
    return _decode_frames(lib().sogrand_decode_product, code, llr_ch, list_max, query_cap, max_iter, alpha,
                          early_stop, want_app, outputs, stream, list_bler_stop)


def sogrand_decode_product_noalloc(code: Code, llr_ch, list_max=4, query_cap=1000, max_iter=4, alpha=0.5,
                                   early_stop=True, want_app=False, outputs=None, stream=None, list_bler_stop=0.0):
    """sogrand_decode_product with the library's static work buffer (no device allocation by the
    library; the output tensors are allocated here unless supplied in ``outputs``)."""
    return _decode_frames(lib().sogrand_decode_product_noalloc, code, llr_ch, list_max, query_cap, max_iter, alpha,
                          early_stop, want_app, outputs, stream, list_bler_stop)


class Plan:
    """sogrand_plan_create/launch/destroy: a product (or QC-GLDPC) decode of the frames in llr_ch
    (F, n, n), recorded once as a HIP graph; launch() decodes what llr_ch holds then into the
    plan's output tensors (``outputs``, the same dict as sogrand_decode_product returns)."""

    def __init__(self, code: Code, llr_ch, list_max=4, query_cap=1000, max_iter=4, alpha=0.5, early_stop=True,
                 want_app=False, gldpc=False, list_bler_stop=0.0):
        import torch
        if not llr_ch.is_cuda or not llr_ch.is_contiguous() or llr_ch.dim() != 3 or \
                llr_ch.shape[1] != code.n or llr_ch.shape[2] != code.n:
            raise ValueError("llr_ch must be a contiguous CUDA tensor of shape (F, n, n)")
        F, n = llr_ch.shape[0], code.n
        dev, dt = llr_ch.device, llr_ch.dtype
        self.llr_ch, self.code = llr_ch, code
        self.outputs = dict(
            hard=torch.empty((F, n, n), dtype=torch.uint8, device=dev),
            llr_app=torch.empty((F, n, n), dtype=dt, device=dev) if want_app else None,
            success=torch.empty(F, dtype=torch.uint8, device=dev),
            half_iters=torch.empty(F, dtype=torch.int16, device=dev),
            sum_queries=torch.empty(F, dtype=torch.int64, device=dev),
            sum_max_queries=torch.empty(F, dtype=torch.int64, device=dev),
        )
        p = params(list_max=list_max, query_cap=query_cap, alpha=alpha, max_iter=max_iter,
                   early_stop=early_stop, precision=_precision_of(llr_ch), list_bler_stop=list_bler_stop)
        o = self.outputs
        h = ctypes.c_void_p()
        _check(lib().sogrand_plan_create(code.handle, ctypes.byref(p), F, 1 if gldpc else 0, _ptr(llr_ch),
                                         _ptr(o["hard"]), _ptr(o["llr_app"]), _ptr(o["success"]),
                                         _ptr(o["half_iters"]), _ptr(o["sum_queries"]), _ptr(o["sum_max_queries"]),
                                         ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(lib().sogrand_plan_launch(self.handle, _stream(stream)))
        return self.outputs

    def close(self):
        if getattr(self, "handle", None):
            lib().sogrand_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def sogrand_decode_gldpc(code: Code, llr_ch, list_max=4, query_cap=1000, max_iter=20, alpha=0.6,
                         early_stop=True, want_app=False, outputs=None, stream=None, list_bler_stop=0.0):
    """The same loop over QC-GLDPC frames llr_ch (F, n, n), element [j, c] being variable node
    j*n + c (column c of block j of the adjacency matrix); returns a dict of tensors."""
    return _decode_frames(lib().sogrand_decode_gldpc, code, llr_ch, list_max, query_cap, max_iter, alpha,
                          early_stop, want_app, outputs, stream, list_bler_stop)


def _decode_frames(fn, code, llr_ch, list_max, query_cap, max_iter, alpha, early_stop, want_app, outputs,
                   stream, list_bler_stop):
    import torch
    if not llr_ch.is_cuda or not llr_ch.is_contiguous() or llr_ch.dim() != 3 or \
            llr_ch.shape[1] != code.n or llr_ch.shape[2] != code.n:
        raise ValueError("llr_ch must be a contiguous CUDA tensor of shape (F, n, n)")
    F, n = llr_ch.shape[0], code.n
    dev, dt = llr_ch.device, llr_ch.dtype
    out = dict(
        hard=torch.empty((F, n, n), dtype=torch.uint8, device=dev),
        llr_app=torch.empty((F, n, n), dtype=dt, device=dev) if want_app else None,
        success=torch.empty(F, dtype=torch.uint8, device=dev),
        half_iters=torch.empty(F, dtype=torch.int16, device=dev),
        sum_queries=torch.empty(F, dtype=torch.int64, device=dev),
        sum_max_queries=torch.empty(F, dtype=torch.int64, device=dev),
    )
    if outputs:
        out.update(outputs)
    p = params(list_max=list_max, query_cap=query_cap, alpha=alpha, max_iter=max_iter,
               early_stop=early_stop, precision=_precision_of(llr_ch), list_bler_stop=list_bler_stop)
    _check(fn(
        code.handle, ctypes.byref(p), F, _ptr(llr_ch), _ptr(out["hard"]), _ptr(out["llr_app"]),
        _ptr(out["success"]), _ptr(out["half_iters"]), _ptr(out["sum_queries"]),
        _ptr(out["sum_max_queries"]), _stream(stream)))
    return out


def sched(waves_per_group=None, frames_per_group=None, steal_chunk=None, groups_per_cu=None):
    """Launch shape of the batched kernel; unspecified fields take the library default."""
    sc = sogrand_sched_t()
    lib().sogrand_sched_default(ctypes.byref(sc))
    for k, v in (("waves_per_group", waves_per_group), ("frames_per_group", frames_per_group),
                 ("steal_chunk", steal_chunk), ("groups_per_cu", groups_per_cu)):
        if v is not None:
            setattr(sc, k, int(v))
    return sc


def pack_frames(frames):
    """Packs a list of (n, n) LLR tensors into one flat tensor plus element offsets (int64)."""
    import torch
    sizes = [f.numel() for f in frames]
    offs = [0]
    for z in sizes[:-1]:
        offs.append(offs[-1] + z)
    flat = torch.cat([f.reshape(-1) for f in frames])
    return flat, torch.tensor(offs, dtype=torch.int64, device=flat.device)


def sogrand_decode_batched(codes, frame_code, frame_offset, llr, list_max=4, query_cap=1000, max_iter=4,
                           alpha=0.5, early_stop=True, sched_=None, outputs=None, stream=None, list_bler_stop=0.0,
                           want_app=False):
    """Batched decode of product frames of mixed codes in one persistent launch.

    codes: list of Code; frame_code: (F,) uint8 CUDA tensor of indices into codes;
    frame_offset: (F,) int64 CUDA tensor of element offsets into llr (flat CUDA
    tensor, float64 or float32).  Returns a dict with hard (flat uint8 like llr),
    success, half_iters, sum_queries, sum_max_queries and status; with want_app also
    llr_app (flat, like llr).
    """
    return _batched(lib().sogrand_decode_batched, codes, frame_code, frame_offset, llr, list_max, query_cap,
                    max_iter, alpha, early_stop, sched_, outputs, stream, list_bler_stop, want_app)


def sogrand_decode_batched_gldpc(codes, frame_code, frame_offset, llr, list_max=4, query_cap=1000, max_iter=20,
                                 alpha=0.6, early_stop=True, sched_=None, outputs=None, stream=None,
                                 list_bler_stop=0.0, want_app=False):
    """sogrand_decode_batched for QC-GLDPC frames (laid out by variable node, as for
    sogrand_decode_gldpc)."""
    return _batched(lib().sogrand_decode_batched_gldpc, codes, frame_code, frame_offset, llr, list_max, query_cap,
                    max_iter, alpha, early_stop, sched_, outputs, stream, list_bler_stop, want_app)


def _batched(fn, codes, frame_code, frame_offset, llr, list_max, query_cap, max_iter, alpha, early_stop, sched_,
             outputs, stream, list_bler_stop, want_app=False):
    import torch
    if not (llr.is_cuda and llr.is_contiguous() and llr.dim() == 1):
        raise ValueError("llr must be a contiguous 1-D CUDA tensor")
    F = frame_code.shape[0]
    if frame_offset.shape[0] != F or frame_code.dtype != torch.uint8 or frame_offset.dtype != torch.int64:
        raise ValueError("frame_code must be uint8 and frame_offset int64, one per frame")
    dev = llr.device
    out = dict(
        hard=torch.empty(llr.shape, dtype=torch.uint8, device=dev),
        llr_app=torch.empty_like(llr) if want_app else None,
        success=torch.empty(F, dtype=torch.uint8, device=dev),
        half_iters=torch.empty(F, dtype=torch.int16, device=dev),
        sum_queries=torch.empty(F, dtype=torch.int64, device=dev),
        sum_max_queries=torch.empty(F, dtype=torch.int64, device=dev),
        status=torch.zeros(1, dtype=torch.int32, device=dev),
    )
    if outputs:
        out.update(outputs)
    handles = (ctypes.c_void_p * len(codes))(*[c.handle for c in codes])
    p = params(list_max=list_max, query_cap=query_cap, alpha=alpha, max_iter=max_iter,
               early_stop=early_stop, precision=_precision_of(llr), list_bler_stop=list_bler_stop)
    # no shape: the library's tuned shape for this kind of batch, else its default
    _check(fn(
        handles, len(codes), ctypes.byref(p), F, _ptr(frame_code), _ptr(frame_offset), llr.numel(),
        _ptr(llr), _ptr(out["hard"]), _ptr(out.get("llr_app")), _ptr(out["success"]), _ptr(out["half_iters"]),
        _ptr(out["sum_queries"]),
        _ptr(out["sum_max_queries"]), _ptr(out["status"]), None if sched_ is None else ctypes.byref(sched_),
        _stream(stream)))
    return out


def sched_tune(codes, frame_code, frame_offset, llr, list_max=4, query_cap=1000, max_iter=4, alpha=0.5,
               early_stop=True, list_bler_stop=0.0, gldpc=False, stream=None):
    """The library's launch-shape tuner on a sample batch (arguments as for sogrand_decode_batched);
    returns (shape, milliseconds).  The shape is also recorded for later calls without one."""
    if not (llr.is_cuda and llr.is_contiguous() and llr.dim() == 1):
        raise ValueError("llr must be a contiguous 1-D CUDA tensor")
    handles = (ctypes.c_void_p * len(codes))(*[c.handle for c in codes])
    p = params(list_max=list_max, query_cap=query_cap, alpha=alpha, max_iter=max_iter,
               early_stop=early_stop, precision=_precision_of(llr), list_bler_stop=list_bler_stop)
    best, ms = sogrand_sched_t(), ctypes.c_float()
    _check(lib().sogrand_sched_tune(1 if gldpc else 0, handles, len(codes), ctypes.byref(p), frame_code.shape[0],
                                    _ptr(frame_code), _ptr(frame_offset), llr.numel(), _ptr(llr),
                                    ctypes.byref(best), ctypes.byref(ms), _stream(stream)))
    return best, ms.value


def sched_table_save(path: str):
    _check(lib().sogrand_sched_table_save(os.fsencode(path)))


def sched_table_load(path: str) -> int:
    """Adds a saved table of tuned shapes; returns the number of entries read."""
    rc = lib().sogrand_sched_table_load(os.fsencode(path))
    if rc < 0:
        _check(rc)
    return rc


def sched_table_clear():
    lib().sogrand_sched_table_clear()


def measure_valu_rate(kind: int = 0, stream=None) -> float:
    """The device's measured VALU issue rate in lane-operations per second for one instruction
    kind: 0 integer XOR/ADD (the measured counterpart of the ALU roofline's derived peak), 1 binary64
    FMA, 2 integer bit-field extract and shift-add."""
    rate, ms = ctypes.c_double(), ctypes.c_double()
    _check(lib().sogrand_measure_valu_rate(int(kind), ctypes.byref(rate), ctypes.byref(ms), _stream(stream)))
    return rate.value


def sogrand_clock_ns() -> int:
    """The library's clock (CLOCK_MONOTONIC, ns), the clock of serving timestamps."""
    return int(lib().sogrand_clock_ns())


class Server:
    """A serving instance: continuous batching of product-frame decode requests.

    Frames are submitted from host memory (numpy arrays of shape (n, n) in the
    server's precision) and results are taken with poll().
    """

    def __init__(self, hbm_budget_bytes, list_max=4, query_cap=1000, max_iter=4, alpha=0.5, early_stop=True,
                 precision=SOGRAND_F32, list_bler_stop=0.0, export_app=False):
        self._h = ctypes.c_void_p()
        self.precision = precision
        self.export_app = bool(export_app)
        p = params(list_max=list_max, query_cap=query_cap, alpha=alpha, max_iter=max_iter,
                   early_stop=early_stop, precision=precision, list_bler_stop=list_bler_stop)
        _check(lib().sogrand_serve_create(ctypes.byref(p), int(hbm_budget_bytes),
                                          SOGRAND_SERVE_APP if export_app else 0, ctypes.byref(self._h)))

    def submit(self, code: Code, llr_host, tag: int = 0):
        """Submits one frame; returns its request id, or None if no slot is free (retry after poll)."""
        import numpy as np
        want = np.float64 if self.precision == SOGRAND_F64 else np.float32
        if llr_host.dtype != want or not llr_host.flags.c_contiguous or llr_host.size != code.n * code.n:
            raise ValueError(f"llr_host must be a C-contiguous {want.__name__} array of n*n elements")
        rid = ctypes.c_uint64()
        rc = lib().sogrand_serve_submit(self._h, code.handle, ctypes.c_void_p(llr_host.ctypes.data),
                                        int(tag), ctypes.byref(rid))
        if rc == SOGRAND_EAGAIN:
            return None
        _check(rc)
        return rid.value

    def poll(self, max_results=256, timeout_ns=0, want_hard=True):
        """Finished requests as a list of dicts (hard: (n, n) uint8 numpy array when want_hard;
        llr_app: (n, n) numpy array of the server's precision when the server exports it)."""
        import numpy as np
        res = (sogrand_result_t * max_results)()
        hard = np.empty(max_results * 128 * 128, dtype=np.uint8) if want_hard else None
        app = None
        if self.export_app:
            app = np.empty(max_results * 128 * 128, dtype=np.float64 if self.precision == SOGRAND_F64 else np.float32)
        nres = ctypes.c_size_t()
        rc = lib().sogrand_serve_poll(self._h, res, max_results, ctypes.byref(nres),
                                      None if hard is None else ctypes.c_void_p(hard.ctypes.data),
                                      None if app is None else ctypes.c_void_p(app.ctypes.data), int(timeout_ns))
        if rc in (SOGRAND_ETIMEDOUT, SOGRAND_ENOTFOUND):
            return []
        _check(rc)
        out = []
        for i in range(nres.value):
            r = res[i]
            d = dict(request_id=r.request_id, user_tag=r.user_tag, status=r.status, success=r.success,
                     half_iters=r.half_iters, n=r.n, queries=r.queries, t_submit_ns=r.t_submit_ns,
                     t_admit_ns=r.t_admit_ns, t_done_ns=r.t_done_ns)
            nn = r.n * r.n
            if hard is not None:
                d["hard"] = hard[r.hard_offset:r.hard_offset + nn].reshape(r.n, r.n).copy()
            if app is not None:
                d["llr_app"] = app[r.hard_offset:r.hard_offset + nn].reshape(r.n, r.n).copy()
            out.append(d)
        return out

    def replay(self, codes, req_code, req_offset, llr_host, arrival_ns, t0_ns):
        """Submits a trace open-loop (see sogrand_serve_replay); returns the refused-attempt count.
        Blocks; poll from another thread meanwhile (the call releases the GIL)."""
        import numpy as np
        req_code = np.ascontiguousarray(req_code, dtype=np.uint8)
        req_offset = np.ascontiguousarray(req_offset, dtype=np.uint64)
        arrival_ns = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
        want = np.float64 if self.precision == SOGRAND_F64 else np.float32
        if llr_host.dtype != want or not llr_host.flags.c_contiguous:
            raise ValueError(f"llr_host must be a C-contiguous {want.__name__} array")
        handles = (ctypes.c_void_p * len(codes))(*[c.handle for c in codes])
        retries = ctypes.c_uint64()
        _check(lib().sogrand_serve_replay(
            self._h, handles, len(codes), req_code.shape[0], ctypes.c_void_p(req_code.ctypes.data),
            ctypes.c_void_p(req_offset.ctypes.data), ctypes.c_void_p(llr_host.ctypes.data), llr_host.size,
            ctypes.c_void_p(arrival_ns.ctypes.data), int(t0_ns), ctypes.byref(retries)))
        return retries.value

    def stats(self):
        st = sogrand_serve_stats_t()
        _check(lib().sogrand_serve_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().sogrand_serve_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
