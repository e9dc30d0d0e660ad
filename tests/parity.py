"""Shared comparison helpers for the GPU-vs-oracle parity tests.

Tolerances (from the arithmetic, stated once here):
  * query numbers, query counts, list sizes, error patterns, hard decisions,
    product counters: bit-exact;
  * LLRs, binary64 path: |dL| <= max(1e-12 max(1, |L|), 64 eps kappa) with
    eps = 2^-52 and kappa = (parity-class mass) / (not-found mass), the
    condition number of M = class mass - queried mass (the subtraction in
    Corollary 1 loses log2(kappa) bits whichever side computes it);
  * LLRs, binary32 storage: the oracle gets the same binary32-rounded inputs;
    |dL| <= max(1e-4, 64 eps kappa + 2^-23 |L|) (output rounding to binary32);
  * APPs of found codewords and P(not found): |dP| <= 1e-12 + 64 eps kappa.
A hard decision may differ only where the oracle's |L_APP| is inside the LLR
tolerance (the sign is then not determined by the arithmetic).
"""
import numpy as np

EPS = 2.0 ** -52


def kappa(diag):
    """Condition number of the not-found mass per word from the oracle's diagnostics."""
    Ppar, M = diag[:, 3], diag[:, 2]
    with np.errstate(divide="ignore"):
        return np.where(M > 0, Ppar / np.maximum(M, 1e-300), np.inf)


def llr_tolerance(ref_llr, kap, f32=False):
    k = np.asarray(kap, dtype=np.float64)[:, None] if np.ndim(kap) else kap
    kterm = np.where(np.isfinite(k), 64 * EPS * k, np.inf)
    if f32:
        return np.maximum(1e-4, kterm + 2.0 ** -23 * np.abs(ref_llr))
    return np.maximum(1e-12 * np.maximum(1.0, np.abs(ref_llr)), kterm)


def compare_component(gpu, ref, f32=False, label=""):
    """gpu: dict of numpy arrays from the library; ref: oracle dict (with diag and found_z)."""
    W = ref["n_queries"].shape[0]
    L = ref["found_q"].shape[1]
    np.testing.assert_array_equal(gpu["n_queries"].astype(np.int64), ref["n_queries"].astype(np.int64), err_msg=label)
    np.testing.assert_array_equal(gpu["n_found"].astype(np.int64), ref["n_found"].astype(np.int64), err_msg=label)
    np.testing.assert_array_equal(gpu["found_q"].astype(np.int64), ref["found_q"].astype(np.int64), err_msg=label)
    if gpu.get("found_z") is not None:
        np.testing.assert_array_equal(gpu["found_z"], ref["found_z"], err_msg=label)
    kap = kappa(ref["diag"])
    tol = llr_tolerance(ref["llr_app"], kap, f32)
    d_app = np.abs(gpu["llr_app"].astype(np.float64) - ref["llr_app"])
    bad = d_app > tol
    assert not bad.any(), f"{label}: {bad.sum()} LLRs off, worst {d_app[bad].max()} (tol {tol[bad].min()})"
    d_ext = np.abs(gpu["llr_ext"].astype(np.float64) - ref["llr_ext"])
    assert not (d_ext > tol + 1e-12 * np.abs(ref["llr_app"])).any(), label
    amb = np.abs(ref["llr_app"]) <= tol
    hd = gpu["hard"] != ref["hard"]
    assert not (hd & ~amb).any(), f"{label}: {int((hd & ~amb).sum())} hard decisions differ"
    ptol = 1e-12 + np.where(np.isfinite(kap), 64 * EPS * kap, np.inf)
    dpf = np.abs(gpu["p_notfound"] - ref["p_notfound"])
    assert not (dpf > ptol).any(), f"{label}: P_nf off by {dpf.max()}"
    dp = np.abs(gpu["p_found"] - ref["p_found"])
    assert not (dp > ptol[:, None]).any(), f"{label}: P_i off by {dp.max()}"
    return dict(words=W, max_dllr=float(d_app.max()) if d_app.size else 0.0,
                kappa_branch=float(np.mean(np.isfinite(kap) & (64 * EPS * kap > 1e-12))))
