"""CPU oracle for SOGRAND decoding -- TEST INFRASTRUCTURE ONLY.

The oracle (``sogrand_oracle.c``) is a plain sequential C implementation of
soft-output GRAND list decoding and of block-turbo decoding of product codes
and QC-GLDPC codes, written from the paper's definitions (arXiv 2310.10737:
Corollary 1, eq. (LLRi), the block turbo decoding steps, the QC-GLDPC adjacency
matrix of the performance evaluation).  Only ``tests/``, the package smoke check and the
benchmark's ``cpu_baseline`` leg may import it.  It shares no code with the GPU
library and never imports it.

This module only marshals numpy arrays into the C library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sogrand_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math: IEEE semantics are required)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SRC,
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.oracle_order.restype = ctypes.c_long
        L.oracle_order.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, ctypes.c_int, P, P]
        L.oracle_code_is_even.restype = ctypes.c_int
        L.oracle_code_is_even.argtypes = [ctypes.c_int, ctypes.c_int, P]
        L.oracle_decode_component.restype = ctypes.c_int
        L.oracle_decode_component.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_long, P,
                                              ctypes.c_int, ctypes.c_long, ctypes.c_double] + [P] * 10
        for fn in (L.oracle_decode_product, L.oracle_decode_gldpc):
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_long, P,
                           ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                           ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, P, ctypes.c_int]
        L.oracle_vnode.restype = ctypes.c_int
        L.oracle_vnode.argtypes = [ctypes.c_int] * 5
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _hcols(code):
    return np.ascontiguousarray(np.array(code.hcols, dtype=np.uint64))


def order(n: int, parity: int, max_q: int, wcols: int = 32):
    """First max_q patterns (tuples of ranks) of the query order.

    parity: 0 = even-weight patterns, 1 = odd-weight, -1 = all weights.
    """
    ranks = np.zeros((max_q, wcols), dtype=np.uint8)
    w = np.zeros(max_q, dtype=np.uint8)
    cnt = lib().oracle_order(n, parity, max_q, wcols, _p(ranks), _p(w))
    if cnt < 0:
        raise ValueError("pattern wider than wcols")
    return [tuple(int(x) for x in ranks[t, :w[t]]) for t in range(cnt)]


def code_is_even(code) -> bool:
    return bool(lib().oracle_code_is_even(code.n, code.k, _p(_hcols(code))))


def decode_component(code, llr, list_max: int = 4, qcap: int = 1000, want_z: bool = False,
                     want_diag: bool = False, pstop: float = 0.0):
    """SISO SOGRAND decode of each row of llr (W, n) float64 (lambda = L_Ch + L_A).

    pstop > 0 ends a word's search once the predicted list-BLER of the list found so
    far is below pstop.  diag (want_diag): per word p(0|r), the tested mass, the
    not-found mass M, the parity-class mass, and 1.0 if the search tested every
    pattern of the class (M is then exactly 0)."""
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    W, n = llr.shape
    assert n == code.n
    out = dict(
        llr_app=np.zeros((W, n)), llr_ext=np.zeros((W, n)), hard=np.zeros((W, n), np.uint8),
        n_queries=np.zeros(W, np.uint32), n_found=np.zeros(W, np.int32),
        found_q=np.zeros((W, list_max), np.uint32), p_found=np.zeros((W, list_max)),
        p_notfound=np.zeros(W),
        found_z=np.zeros((W, list_max, n), np.uint8) if want_z else None,
        diag=np.zeros((W, 5)) if want_diag else None,
    )
    rc = lib().oracle_decode_component(
        code.n, code.k, _p(_hcols(code)), W, _p(llr), list_max, qcap, float(pstop),
        _p(out["llr_app"]), _p(out["llr_ext"]), _p(out["hard"]), _p(out["n_queries"]),
        _p(out["n_found"]), _p(out["found_q"]), _p(out["p_found"]), _p(out["p_notfound"]),
        _p(out["found_z"]), _p(out["diag"]))
    if rc:
        raise ValueError("oracle_decode_component rejected its arguments")
    return out


def _two_family(fn, name, code, llr_ch, list_max, qcap, max_iter, alpha, early_stop, store_f32, want_app,
                nthreads, pstop, want_last_diag=False):
    llr_ch = np.ascontiguousarray(llr_ch, dtype=np.float64)
    F, n, n2 = llr_ch.shape
    assert n == n2 == code.n
    out = dict(
        hard=np.zeros((F, n, n), np.uint8), llr_app=np.zeros((F, n, n)) if want_app else None,
        success=np.zeros(F, np.uint8), half_iters=np.zeros(F, np.uint16),
        sum_queries=np.zeros(F, np.uint64), sum_max_queries=np.zeros(F, np.uint64),
        last_diag=np.zeros((F, n, 5)) if want_last_diag else None,
        kappa_max=np.zeros(F) if want_last_diag else None,
    )
    rc = fn(code.n, code.k, _p(_hcols(code)), F, _p(llr_ch), list_max, qcap, float(pstop), max_iter, alpha,
            int(early_stop), int(store_f32), _p(out["hard"]), _p(out["llr_app"]), _p(out["success"]),
            _p(out["half_iters"]), _p(out["sum_queries"]), _p(out["sum_max_queries"]), _p(out["last_diag"]),
            _p(out["kappa_max"]), nthreads)
    if rc:
        raise ValueError(f"{name} rejected its arguments")
    return out


def decode_product(code, llr_ch, list_max: int = 4, qcap: int = 1000, max_iter: int = 4,
                   alpha: float = 0.5, early_stop: bool = True, store_f32: bool = False,
                   want_app: bool = False, nthreads: int = 1, pstop: float = 0.0, want_last_diag: bool = False):
    """Block-turbo decode of product-code frames llr_ch (F, n, n) float64, row-major.

    want_last_diag: also return last_diag (F, n, 5), decode_component's diag of each word of
    the frame's last half-iteration (rows after an odd, columns after an even count), and
    kappa_max (F,), the largest condition number class mass / not-found mass over every word
    the frame decoded."""
    return _two_family(lib().oracle_decode_product, "oracle_decode_product", code, llr_ch, list_max, qcap,
                       max_iter, alpha, early_stop, store_f32, want_app, nthreads, pstop, want_last_diag)


def decode_gldpc(code, llr_ch, list_max: int = 4, qcap: int = 1000, max_iter: int = 20,
                 alpha: float = 0.6, early_stop: bool = True, store_f32: bool = False,
                 want_app: bool = False, nthreads: int = 1, pstop: float = 0.0, want_last_diag: bool = False):
    """The same loop over QC-GLDPC frames llr_ch (F, n, n) float64: element [j, c] is variable
    node j*n + c (column c of block j of the adjacency matrix)."""
    return _two_family(lib().oracle_decode_gldpc, "oracle_decode_gldpc", code, llr_ch, list_max, qcap,
                       max_iter, alpha, early_stop, store_f32, want_app, nthreads, pstop, want_last_diag)


def vnode(topo: int, n: int, fam: int, line: int, j: int) -> int:
    """Variable node of bit j of component word `line` of family `fam` (topo 0: product code,
    rows then columns; topo 1: QC-GLDPC, first then second block row)."""
    v = lib().oracle_vnode(topo, n, fam, line, j)
    if v < 0:
        raise ValueError("oracle_vnode rejected its arguments")
    return v


def forney_app(llr, found_z, n_found):
    """Forney's approximation of the probability that each list codeword is correct (eq.
    (missingterm), section "Background on SO"): its likelihood divided by the sum of the list's
    likelihoods, the codewords outside the list counted as zero.

    With BPSK over AWGN and lambda = 2r/sigma^2, the likelihood of the codeword y XOR z (y the hard
    decision) over that of y is exp(-sum over i with z_i = 1 of |lambda_i|), which is what is summed
    here.  llr (W, n), found_z (W, L, n) error patterns, n_found (W,).  Returns (W, L) float64, zero
    past n_found; a word whose list is empty gets a row of NaN (the approximation needs a list).
    """
    a = np.abs(np.asarray(llr, dtype=np.float64))
    z = np.asarray(found_z).astype(np.float64)
    W, L, n = z.shape
    nf = np.asarray(n_found).astype(np.int64)
    valid = np.arange(L)[None, :] < nf[:, None]
    loglik = -(z * a[:, None, :]).sum(axis=2)
    top = np.where(valid, loglik, -np.inf).max(axis=1, keepdims=True)
    with np.errstate(invalid="ignore"):
        lik = np.where(valid, np.exp(loglik - top), 0.0)
        return lik / lik.sum(axis=1, keepdims=True)


def forney_list_bler(llr, found_z, n_found, lprime: int):
    """Predicted probability that the transmitted codeword is not among the first lprime entries of
    the list, by Forney's approximation over the whole list (the paper's Fig. 2 uses a list of 5 to
    predict the error of the first 4): one minus their summed forney_app."""
    p = forney_app(llr, found_z, n_found)
    return np.maximum(1.0 - p[:, :lprime].sum(axis=1), 0.0)
