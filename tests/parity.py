"""Shared comparison helpers for the GPU-vs-oracle parity tests.

Tolerances (from the arithmetic, stated once here):
  * query numbers, query counts, list sizes, error patterns, hard decisions,
    product counters: bit-exact;
  * LLRs, binary64 path: |dL| <= max(1e-12 max(1, |L|), 64 eps kappa) with
    eps = 2^-52 and kappa = (parity-class mass) / (not-found mass), the
    condition number of M = class mass - queried mass (the subtraction in
    Corollary 1 loses log2(kappa) bits whichever side computes it).  A word whose
    search tested its whole class has M = 0 exactly on both sides (no subtraction),
    so kappa = 0 there.  The kappa term is not scaled down by P_nf: on a bit where
    every list codeword agrees, one of the two sums of eq. (LLRi) is P_nf times the
    soft input alone, so L moves by the relative error of P_nf, which is that of M;
  * LLRs, binary32 storage: the oracle gets the same binary32-rounded inputs;
    |dL| <= max(1e-4, 64 eps kappa + 2^-23 |L|) (output rounding to binary32);
  * APPs of found codewords and P(not found): |dP| <= 1e-12 + 64 eps kappa.
A hard decision may differ only where the oracle's |L_APP| is inside the LLR
tolerance (the sign is then not determined by the arithmetic).
"""
import numpy as np

EPS = 2.0 ** -52


def kappa(diag):
    """Condition number of the not-found mass per word from the oracle's diagnostics: 0 when
    the class was exhausted (M = 0 exactly), inf when M is not positive otherwise (M is then
    below the rounding of the subtraction, and the LLRs that depend on it are undetermined)."""
    Ppar, M, exhausted = diag[..., 3], diag[..., 2], diag[..., 4] > 0
    with np.errstate(divide="ignore"):
        k = np.where(M > 0, Ppar / np.maximum(M, 1e-300), np.inf)
    return np.where(exhausted, 0.0, k)


def llr_tolerance(ref_llr, kap, f32=False):
    k = np.asarray(kap, dtype=np.float64)[..., None] if np.ndim(kap) else kap
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


def last_pass_kappa(ref, topo=0):
    """kappa of the last half-iteration's word holding each element of the frames (F, n, n).

    ref: oracle product or QC-GLDPC output with last_diag.  Element [j][c] of a product frame
    lies in row j and column c; of a QC-GLDPC frame (variable node j*n + c) in word c of the
    first block row and word (c - j) mod n of the second."""
    ld = ref["last_diag"]
    F, n, _ = ld.shape
    kw = kappa(ld)
    rows_last = (ref["half_iters"].astype(np.int64) % 2) == 1
    j = np.arange(n)[:, None]
    c = np.arange(n)[None, :]
    if topo == 0:
        w_first, w_second = np.broadcast_to(j, (n, n)), np.broadcast_to(c, (n, n))
    else:
        w_first, w_second = np.broadcast_to(c, (n, n)), (c - j) % n
    idx = np.where(rows_last[:, None, None], w_first[None], w_second[None]).reshape(F, -1)
    return np.take_along_axis(kw, idx, axis=1).reshape(F, n, n)


def compare_product(g, r, f32=False, label="", topo=0):
    """Product or QC-GLDPC frames, GPU (g) against the oracle (r, decoded with want_last_diag).

    Bit-exact: success, half-iterations, sum of queries, sum of per-half maxima, hard decision.
    L_APP, element by element, within the product-level form of the bound above:
        |dL| <= max(1e-12 max(1, |L|), 64 eps kappa_traj)          (binary64)
        |dL| <= max(1e-4, 64 eps kappa_traj + 2^-23 |L|)            (binary32 storage)
    where kappa_traj is the largest condition number of a not-found mass over every word the
    oracle decoded in that frame: the last pass adds its own word's kappa term, and an earlier
    pass's kappa-sized error reaches the last pass's inputs through L_A = alpha L_E.  Returns
    the worst ratio to the bound with the last pass's own kappa in place of kappa_traj, the
    fraction of elements beyond that tighter bound, and the kappa-branch fractions."""
    for key in ("success", "half_iters", "sum_queries", "sum_max_queries"):
        if g.get(key) is not None:   # the served form reports no per-half maxima
            np.testing.assert_array_equal(g[key].astype(np.int64), r[key].astype(np.int64), err_msg=f"{label}: {key}")
    np.testing.assert_array_equal(g["hard"].reshape(r["hard"].shape), r["hard"], err_msg=label)
    stats = dict(frames=int(r["success"].shape[0]))
    if g.get("llr_app") is None or r.get("llr_app") is None:
        return stats
    ref = r["llr_app"]
    d = np.abs(g["llr_app"].astype(np.float64).reshape(ref.shape) - ref)
    kl = last_pass_kappa(r, topo)
    kt = np.broadcast_to(r["kappa_max"][:, None, None], ref.shape)
    with np.errstate(invalid="ignore", over="ignore"):
        if f32:
            tol_last = np.maximum(1e-4, 64 * EPS * kl + 2.0 ** -23 * np.abs(ref))
            tol = np.maximum(1e-4, 64 * EPS * kt + 2.0 ** -23 * np.abs(ref))
        else:
            base = 1e-12 * np.maximum(1.0, np.abs(ref))
            tol_last = np.maximum(base, 64 * EPS * kl)
            tol = np.maximum(base, 64 * EPS * kt)
        tol = np.maximum(tol, tol_last)
        ratio_last = np.where(np.isfinite(tol_last), d / tol_last, 0.0)
    bad = d > tol
    stats.update(worst_ratio_last=float(ratio_last.max()), frac_beyond_last=float(np.mean(ratio_last > 1.0)),
                 kappa_branch_last=float(np.mean(64 * EPS * kl > 1e-12)),
                 kappa_branch_traj=float(np.mean(64 * EPS * kt > 1e-12)),
                 frames_kappa_inf=int(np.sum(~np.isfinite(r["kappa_max"]))), max_dllr=float(d.max()))
    print(f"[parity] {label}: worst |dL|/bound(last pass) {stats['worst_ratio_last']:.3g}, beyond it "
          f"{stats['frac_beyond_last']:.2e}; kappa branch {stats['kappa_branch_last']:.3f} (last) "
          f"{stats['kappa_branch_traj']:.3f} (trajectory); max |dL| {stats['max_dllr']:.3g}", flush=True)
    assert not bad.any(), (f"{label}: {int(bad.sum())} L_APP beyond the bound, worst {d[bad].max():.3e} "
                           f"(bound {tol[bad].min():.3e})")
    return stats
