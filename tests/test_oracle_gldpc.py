"""Pins of the oracle's QC-GLDPC decoding (the (n^2, n^2 - 2n(n-k)) codes of the performance
evaluation, adjacency matrix [I(0) ... I(0); I(0) I(1) ... I(n-1)]).

What fixes the oracle here, independently of its own arithmetic:
* the adjacency matrix's shape: every variable node lies on exactly one check node of each block
  row, and bit j of every check node comes from block j;
* the code is quasi-cyclic: rotating every block by one position maps check nodes onto check nodes;
* the product-code case of the same index function has dimension k^2, and the QC-GLDPC case has at
  least the paper's design dimension n^2 - 2n(n-k), equal to that of the input generator's own,
  separately written construction, whose codewords satisfy every oracle check node;
* the decoder commutes with adding a codeword: flipping the LLR signs along a codeword flips the
  hard decision by it and leaves every query count and |L_APP| unchanged;
* noiseless frames decode in the first half-iteration.
"""
import numpy as np
import pytest

import oracle
import synth

GLDPC = 1


def check_nodes(n, topo):
    """(2, n, n) variable node of bit j of check node `line` of each family, from the oracle."""
    return np.array([[[oracle.vnode(topo, n, fam, line, j) for j in range(n)] for line in range(n)]
                     for fam in (0, 1)])


def rank_gf2(rows):
    basis = []
    for r in rows:
        for piv, b in basis:
            if (r >> piv) & 1:
                r ^= b
        if r:
            basis.append((r.bit_length() - 1, r))
    return len(basis)


def code_dimension(code, topo):
    cn = check_nodes(code.n, topo)
    H = code.H()
    rows = []
    for fam in (0, 1):
        for line in range(code.n):
            for q in range(code.r):
                v = 0
                for j in range(code.n):
                    if H[q, j]:
                        v |= 1 << int(cn[fam, line, j])
                rows.append(v)
    return code.n * code.n - rank_gf2(rows)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_adjacency_shape(n):
    cn = check_nodes(n, GLDPC)
    for fam in (0, 1):
        # each variable node on exactly one check node of the block row
        assert sorted(cn[fam].ravel().tolist()) == list(range(n * n))
        # bit j of every check node comes from block j
        assert np.all(cn[fam] // n == np.arange(n)[None, :])
    # the first block row is all identities: check node r meets column r of every block
    assert np.all(cn[0] % n == np.arange(n)[:, None])


@pytest.mark.parametrize("n", [16, 32])
def test_quasi_cyclic(n):
    cn = check_nodes(n, GLDPC)
    rot = lambda v: (v // n) * n + (v % n + 1) % n   # noqa: E731  column c -> c + 1 in every block
    for fam in (0, 1):
        images = {frozenset(rot(v) for v in cn[fam, line]) for line in range(n)}
        assert images == {frozenset(cn[fam, line].tolist()) for line in range(n)}
    # the second block row is not the first one again (that would be a repetition, not a GLDPC)
    assert {frozenset(x.tolist()) for x in cn[0]} != {frozenset(x.tolist()) for x in cn[1]}


@pytest.mark.parametrize("nk", [(16, 11), (32, 26)])
def test_dimension(nk):
    code = synth.ebch(*nk)
    n, k = nk
    assert code_dimension(code, 0) == k * k                 # the product code, through the same function
    dim = code_dimension(code, GLDPC)
    assert dim >= n * n - 2 * n * (n - k)                    # the paper's (n^2, n^2 - 2n(n-k))
    g = synth.gldpc(code)
    assert g.dim == dim
    # the generator's codewords satisfy every check node of the oracle's structure
    cn = check_nodes(n, GLDPC)
    u = synth.info_bits(3, np.arange(20, dtype=np.uint64), g.dim)
    cw = (u.astype(np.int64) @ g.G.astype(np.int64)) % 2
    H = code.H().astype(np.int64)
    for fam in (0, 1):
        words = cw[:, cn[fam]]                               # (F, n lines, n bits)
        assert not np.any((words @ H.T) % 2)


def test_noiseless_frames_decode_at_once():
    code = synth.ebch(32, 26)
    g = synth.gldpc(code)
    llr, cw, _ = synth.gldpc_frames(g, 30.0, 4, np.arange(6))
    out = oracle.decode_gldpc(code, llr, 4, 1000, 20, 0.6)
    assert np.all(out["success"] == 1) and np.all(out["half_iters"] == 1)
    np.testing.assert_array_equal(out["hard"], cw)


@pytest.mark.parametrize("stop", [0.0, 1e-5])
def test_codeword_translation(stop):
    code = synth.ebch(32, 26)
    g = synth.gldpc(code)
    llr, _, _ = synth.gldpc_frames(g, 2.25, 5, np.arange(24))
    _, c, _ = synth.gldpc_frames(g, 2.25, 6, np.arange(24))
    flipped = np.where(c == 1, -llr, llr)
    a = oracle.decode_gldpc(code, llr, 4, 2000, 12, 0.6, want_app=True, pstop=stop)
    b = oracle.decode_gldpc(code, flipped, 4, 2000, 12, 0.6, want_app=True, pstop=stop)
    np.testing.assert_array_equal(b["hard"], a["hard"] ^ c)
    for key in ("success", "half_iters", "sum_queries", "sum_max_queries"):
        np.testing.assert_array_equal(b[key], a[key], err_msg=key)
    np.testing.assert_array_equal(b["llr_app"], np.where(c == 1, -a["llr_app"], a["llr_app"]))
    # frames needing several iterations are part of the case
    assert a["half_iters"].max() > 2


def test_planted_wrong_rotation_fails_translation():
    """A structure that is not the code's (here: the second block row rotated the other way for
    the decoder, while the codeword comes from the paper's construction) breaks the symmetry, so the
    translation test above would catch a wrong index function."""
    code = synth.ebch(32, 26)
    g = synth.gldpc(code)
    llr, _, _ = synth.gldpc_frames(g, 2.25, 5, np.arange(8))
    _, c, _ = synth.gldpc_frames(g, 2.25, 6, np.arange(8))
    # mirror the blocks (j -> -j mod n): a codeword of the mirrored code, not of this one
    n = code.n
    cm = c[:, (-np.arange(n)) % n, :]
    flipped = np.where(cm == 1, -llr, llr)
    a = oracle.decode_gldpc(code, llr, 4, 2000, 12, 0.6)
    b = oracle.decode_gldpc(code, flipped, 4, 2000, 12, 0.6)
    assert not np.array_equal(b["hard"], a["hard"] ^ cm)


def test_rejects_bad_arguments():
    code = synth.ebch(32, 26)
    llr = np.zeros((1, 32, 32))
    with pytest.raises(ValueError):
        oracle.decode_gldpc(code, llr, 0, 1000, 20, 0.6)
    with pytest.raises(ValueError):
        oracle.decode_gldpc(code, llr, 4, 1000, 20, 0.6, pstop=2.0)
    with pytest.raises(ValueError):
        oracle.vnode(2, 32, 0, 0, 0)
