"""Pins for the oracle's block-turbo exchange (section "Iterative decoding": L_A = 0, each
half-iteration decodes L_Ch + L_A, then L_A = alpha L_E with L_E = L_APP - L_Ch - L_A) and for
reading R8 (the soft input of eq. (LLRi) is the SISO input L_Ch + L_A).

The expected values never come from the oracle: they are the exact bitwise APP LLRs of the
component code, summed over its whole codebook, and the closed form of Corollary 1 for a list
of one codeword found at the first query.  Each test also checks that the plausible misreadings
(L_A = alpha L_APP, alpha dropped, the soft input taken from L_Ch alone) give values far from
the oracle's, so that the test would fail under any of them.
"""
import functools
import itertools

import numpy as np
import pytest

import oracle
import synth

ALPHA = 0.5


def codebook(code):
    msgs = np.array(list(itertools.product([0, 1], repeat=code.k)), dtype=np.int64)
    return ((msgs @ code.G.astype(np.int64)) & 1).astype(np.uint8)


def exact_app(cb, lam):
    """Bitwise APP LLRs log P(c_i = 0 | lam) / P(c_i = 1 | lam) of every word lam[..., n] of a code
    with codebook cb, under independent bits with LLRs lam: P(c) is proportional to
    exp(sum_j lam_j (1 - 2 c_j) / 2)."""
    s = (lam[..., None, :] * (1.0 - 2.0 * cb)).sum(-1) / 2.0
    s = s - s.max(-1, keepdims=True)
    w = np.exp(s)
    num = (w[..., :, None] * (cb == 0)).sum(-2)
    den = (w[..., :, None] * (cb == 1)).sum(-2)
    return np.log(num) - np.log(den)


@functools.lru_cache(maxsize=None)
def vnode_map(topo, n, fam):
    """(n lines, n bits) array of the variable node of bit j of word `line` of family fam."""
    return np.array([[oracle.vnode(topo, n, fam, line, j) for j in range(n)] for line in range(n)])


def words_of(topo, X, n, fam):
    """(F, n lines, n bits) view of frame array X (F, n, n) as the words of family fam."""
    return X.reshape(X.shape[0], -1)[:, vnode_map(topo, n, fam)]


def frame_of(topo, Wd, n, fam):
    """Inverse of words_of."""
    out = np.empty((Wd.shape[0], n * n), dtype=Wd.dtype)
    out[:, vnode_map(topo, n, fam)] = Wd
    return out.reshape(Wd.shape[0], n, n)


def gf2_nullspace(A):
    """Basis (rows) of the null space of A over GF(2), by Gauss-Jordan elimination."""
    A = (A % 2).astype(np.uint8)
    m, v = A.shape
    piv, r = [], 0
    for c in range(v):
        if r == m:
            break
        rows = np.nonzero(A[r:, c])[0]
        if rows.size == 0:
            continue
        p = r + rows[0]
        A[[r, p]] = A[[p, r]]
        nz = np.nonzero(A[:, c])[0]
        A[nz[nz != r]] ^= A[r]
        piv.append(c)
        r += 1
    basis = []
    for f in (c for c in range(v) if c not in piv):
        x = np.zeros(v, np.uint8)
        x[f] = 1
        for i, c in enumerate(piv):
            x[c] = A[i, f]
        basis.append(x)
    return np.array(basis)


def chain(cb, topo, Lch, n, halves, alpha, a_of_app=False, no_alpha=False):
    """The block-turbo chain with every SISO exact (exhaustive list): returns the last L_APP.
    a_of_app / no_alpha: the misreadings L_A = alpha L_APP and L_A = L_E."""
    LA = np.zeros_like(Lch)
    app = None
    for h in range(1, halves + 1):
        fam = 0 if h & 1 else 1
        lam = words_of(topo, Lch + LA, n, fam)
        app_w = exact_app(cb, lam)
        app = frame_of(topo, app_w, n, fam)
        LE = app - (Lch + LA)
        LA = (alpha if not no_alpha else 1.0) * (app if a_of_app else LE)
    return app


@pytest.mark.parametrize("topo", [0, 1])
@pytest.mark.parametrize("nk,ebn0,iters", [((8, 4), 0.5, 2), ((8, 4), 2.0, 1), ((16, 11), 1.5, 1)])
def test_exchange_with_exact_siso_matches_codebook_chain(topo, nk, ebn0, iters):
    """With a list longer than the codebook every component decode is exact (the class is
    exhausted, M = 0), so 2 * iters half-iterations without early stopping must reproduce the
    chain of exact APPs with L_A = alpha (L_APP - L_Ch - L_A) between passes."""
    code = synth.ebch(*nk)
    n = code.n
    F = 3
    if topo == 0:
        llr, _, _ = synth.product_frames(code, ebn0, 61, np.arange(F))
    else:
        llr, _, _ = synth.gldpc_frames(synth.gldpc(code), ebn0, 61, np.arange(F))
    L, cap = (1 << code.k) + 1, 1 << (n - 1)
    decode = oracle.decode_product if topo == 0 else oracle.decode_gldpc
    out = decode(code, llr, L, cap, iters, alpha=ALPHA, early_stop=False, want_app=True, nthreads=4)
    assert np.all(out["half_iters"] == 2 * iters)
    cb = codebook(code).astype(np.float64)
    want = chain(cb, topo, llr, n, 2 * iters, ALPHA)
    scale = np.maximum(1.0, np.abs(want))
    err = np.abs(out["llr_app"] - want) / scale
    assert err.max() < 1e-10, f"worst relative difference {err.max():.3e}"
    # the misreadings land far away
    for kw in (dict(a_of_app=True), dict(no_alpha=True)):
        alt = chain(cb, topo, llr, n, 2 * iters, ALPHA, **kw)
        assert np.abs(out["llr_app"] - alt).max() > 1e-2, kw


def even_class_mass(rho):
    """Sum over every nonzero even-weight subset z of prod_{i in z} rho_i, by enumeration."""
    n = rho.shape[-1]
    masks = np.arange(1, 1 << n)
    bits = ((masks[:, None] >> np.arange(n)) & 1).astype(bool)
    even = bits.sum(1) % 2 == 0
    bits = bits[even]
    logr = np.log(rho)
    return np.exp(bits.astype(np.float64) @ logr.T).sum(0) if rho.ndim > 1 else np.exp(bits @ logr).sum()


@pytest.mark.parametrize("topo", [0, 1])
@pytest.mark.parametrize("nk", [(8, 4), (16, 11)])
def test_prior_from_siso_input_and_alpha_scaled_extrinsic(topo, nk):
    """Reading R8 and the exchange, with L = 1 and a cap of one query.  The first family's
    words are codewords, the second family's are words of even weight that are not:
      * first pass: each word's hard decision is found at query 1; Corollary 1 gives
        P_1 = 1 / (1 + M phi) and P_nf = M phi / (1 + M phi), with M the mass (relative to
        p(0|r)) of the nonzero patterns of the class (even weights).  In eq. (LLRi) bit i
        then has N_y = P_1 + P_nf / (1 + rho_i) and N_not_y = P_nf rho_i / (1 + rho_i),
        rho_i = exp(-|lambda_i|), so L_E,i = (1 - 2 y_i) ln(1 + (1 + rho_i) / (M phi));
      * second pass: nothing is found, P_nf = 1, so L_APP = lambda = L_Ch + alpha L_E,
        the soft input itself, since the prior of eq. (LLRi) is the SISO input.
    """
    code = synth.ebch(*nk)
    assert code.is_even
    n, k = code.n, code.k
    H = code.H().astype(np.int64)
    # frames whose first-family words are codewords u_l G and whose second-family words have
    # even weight: a linear condition on the messages u (n words x k bits), solved over GF(2)
    v0, v1 = vnode_map(topo, n, 0), vnode_map(topo, n, 1)
    word_of, bit_of = np.empty(n * n, np.int64), np.empty(n * n, np.int64)
    word_of[v0.reshape(-1)] = np.repeat(np.arange(n), n)
    bit_of[v0.reshape(-1)] = np.tile(np.arange(n), n)
    A = np.zeros((n, n * k), np.uint8)
    for line in range(n):
        for v in v1[line]:
            A[line, word_of[v] * k:(word_of[v] + 1) * k] ^= code.G[:, bit_of[v]].astype(np.uint8)
    B = gf2_nullspace(A)
    rng = np.random.default_rng(7 + n + topo)
    frames, F = [], 4
    while len(frames) < F:
        u = (rng.integers(0, 2, size=B.shape[0]) @ B) % 2
        words1 = (u.reshape(n, k).astype(np.int64) @ code.G.astype(np.int64)) % 2
        C = frame_of(topo, words1[None], n, 0)[0]
        words2 = words_of(topo, C[None], n, 1)[0]
        assert np.all(words2.sum(1) % 2 == 0)
        # no second-family word is a codeword, so its first query (the zero pattern) misses
        if np.all(np.any((words2 @ H.T) % 2, axis=1)):
            frames.append(C)
    C = np.stack(frames)
    mag = rng.uniform(0.5, 3.0, size=C.shape)
    Lch = (1.0 - 2.0 * C) * mag
    decode = oracle.decode_product if topo == 0 else oracle.decode_gldpc
    out = decode(code, Lch, 1, 1, 1, alpha=ALPHA, early_stop=False, want_app=True)
    assert np.all(out["half_iters"] == 2) and np.all(out["success"] == 0)
    # closed form of the first pass's extrinsic output, word by word
    w1 = words_of(topo, Lch, n, 0)
    rho = np.exp(-np.abs(w1))
    M = np.stack([even_class_mass(rho[f]) for f in range(F)])          # (F, n words)
    phi = (2.0 ** k - 1.0) / (2.0 ** (n - 1) - 1.0)
    y = (w1 < 0).astype(np.float64)
    LE1 = (1.0 - 2.0 * y) * np.log1p((1.0 + rho) / (M * phi)[..., None])
    LE1 = frame_of(topo, LE1, n, 0)
    want = Lch + ALPHA * LE1
    err = np.abs(out["llr_app"] - want) / np.maximum(1.0, np.abs(want))
    assert err.max() < 1e-12, f"worst relative difference {err.max():.3e}"
    np.testing.assert_array_equal(out["hard"], C)
    # the misreadings: prior from L_Ch alone, alpha dropped, L_A = alpha L_APP
    app1 = Lch + LE1
    for alt in (Lch, Lch + LE1, Lch + ALPHA * app1):
        assert np.abs(out["llr_app"] - alt).max() > 0.1
