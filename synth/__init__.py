"""Seeded synthetic inputs for SOGRAND product-code decoding.

This module is shared by the CPU oracle tests and by the GPU library's tests and
benchmark. It holds *none* of the decoding method's arithmetic: it only builds
codes (parity-check columns, generator, information positions), encodes random
information bits, and passes BPSK symbols through an AWGN channel to make
channel LLRs.

Codes
-----
Extended BCH (eBCH) codes of length n = 2^m.  The paper uses eBCH component
codes throughout its product-code experiments (Sec. "Iterative decoding",
Figs. 5, 7, 8, 12, 13) without fixing the field polynomial, the bit order or
the systematic positions.  This module fixes them:

* primitive polynomials x^3+x+1, x^4+x+1, x^5+x^2+1, x^6+x+1, x^7+x^3+1;
* the cyclic BCH code of length 2^m - 1 with zeros alpha^1, alpha^3, ...,
  alpha^(2t-1) (t = 1 is the Hamming code), encoded systematically as
  c(x) = x^r m(x) + (x^r m(x) mod g(x)): parity in positions 0..r-1, the
  message in positions r..n-2;
* one overall parity bit appended at position n-1 (the even extension of the
  section on even codes: G_{i,n} = sum_j G_{i,j}).

The parity-check matrix H has one column per code bit, stored as an integer
whose bit r is H[r][j]; its rows are alpha^{(2i-1)j} written in the field's
polynomial basis, reduced to full rank, plus the all-ones row.  The decoder's
membership test H c = 0 does not depend on which basis of the dual code is used.

QC-GLDPC codes
--------------
The (n^2, n^2 - 2n(n-k)) quasi-cyclic GLDPC codes of the performance evaluation
have the adjacency matrix with block rows [I(0) ... I(0)] and [I(0) I(1) ...
I(n-1)], I(i) the n x n identity rotated right by i positions (row r of I(i) has
its one in column (r + i) mod n).  Each of its 2n rows is a component code whose
bit j sits in block j.  `gldpc` builds the code's parity-check matrix from that
description and a systematic generator of its null space by Gaussian
elimination; frames are [n][n] arrays whose element [j, c] is variable node
j*n + c.  The design dimension n^2 - 2n(n-k) counts every check as independent;
the null space can be larger (for the [32,26] eBCH component, 646 rather than
640), and its true dimension is used.

Channel
-------
BPSK maps bit 0 to +1 and bit 1 to -1.  With overall rate R and Eb/N0 in dB,
sigma^2 = 1 / (2 R 10^(EbN0/10)), r = x + sigma * N(0,1), and the channel LLR is
L_Ch = log p(r|0)/p(r|1) = 2 r / sigma^2 (the SISO section's definition of L_Ch).

Block Rician fading with QPSK
-----------------------------
The block fading section's channel: a frame of N coded bits is interleaved by a
random permutation (its own for every frame), mapped in pairs (c1, c2) to Gray
QPSK x = Delta (1 - 2 c1) + j Delta (1 - 2 c2) with Delta = 1, and sent as N/2
symbols over t coherence blocks of N_c symbols (N = 2 t N_c).  Block b has
H = sqrt(K/(K+1)) + sqrt(1/(K+1)) H_Ra, H_Ra ~ CN(0, 1) (real and imaginary
parts of variance 1/2, so E|H|^2 = 1), and y = H x + z with z ~ CN(0, 2 sigma^2).
With the coefficient known to the receiver, L(c1) = 2 Delta Re(y h*) / sigma^2 and
L(c2) = 2 Delta Im(y h*) / sigma^2, de-interleaved back to code order.  Eb/N0 sets
sigma^2 = Delta^2 / (2 R Eb/N0), since Es/N0 = Delta^2 E|H|^2 / sigma^2 and a
symbol carries 2R information bits.  Streams: the permutation comes from stream 3
(ranks of its outputs), the fading from stream 2, the noise from stream 1.

Random numbers
--------------
Counter-based SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; constants of Vigna's public-domain splitmix64):
the stream for (seed, frame, stream-id) starts from
    k1 = mix(seed XOR 0xA0761D6478BD642F)
    k2 = mix(k1 XOR frame*0x9E3779B97F4A7C15 XOR stream*0xE7037ED1A0B428DB)
and its i-th output (i = 0, 1, ...) is mix(k2 + (i+1)*0x9E3779B97F4A7C15), all
arithmetic modulo 2^64.  Information bits are the top bit of successive outputs
of stream 0.  Gaussian samples come from stream 1 by Box-Muller on output pairs
(2j, 2j+1): u1 = ((o_2j >> 11) + 1) 2^-53, u2 = (o_2j+1 >> 11) 2^-53,
z_2j = sqrt(-2 ln u1) cos(2 pi u2), z_2j+1 = sqrt(-2 ln u1) sin(2 pi u2).
Any frame can therefore be regenerated alone from (seed, frame).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Code", "ebch", "code_from_generator", "encode", "encode_product",
    "splitmix_stream", "info_bits", "gaussians", "sigma2", "bpsk_awgn_llr",
    "product_frames", "component_words", "PRIM_POLY", "Gldpc", "gldpc", "gldpc_frames",
    "rician_qpsk_llr", "rician_product_frames",
]

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
PRIM_POLY = {3: 0b1011, 4: 0b10011, 5: 0b100101, 6: 0b1000011, 7: 0b10001001}


# ----------------------------------------------------------------------------
# codes
# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Code:
    """A binary linear [n, k] code.

    hcols[j] : int, bit r is H[r][j] (n - k rows, full rank).
    G        : (k, n) uint8 generator, systematic on info_pos.
    info_pos : (k,) positions that carry the information bits.
    is_even  : every codeword has even weight.
    """
    name: str
    n: int
    k: int
    hcols: tuple
    G: np.ndarray
    info_pos: tuple
    is_even: bool

    @property
    def r(self) -> int:
        return self.n - self.k

    def hcols_u64(self) -> np.ndarray:
        return np.array(self.hcols, dtype=np.uint64)

    def hcols_u32(self) -> np.ndarray:
        if self.r > 32:
            raise ValueError("more than 32 parity checks")
        return np.array(self.hcols, dtype=np.uint32)

    def H(self) -> np.ndarray:
        """(n-k, n) uint8 parity-check matrix."""
        h = np.zeros((self.r, self.n), dtype=np.uint8)
        for j, c in enumerate(self.hcols):
            for r in range(self.r):
                h[r, j] = (c >> r) & 1
        return h


def _gf_tables(m: int):
    poly = PRIM_POLY[m]
    q = 1 << m
    exp = [0] * (2 * q)
    x = 1
    for i in range(q - 1):
        exp[i] = x
        x <<= 1
        if x & q:
            x ^= poly
    for i in range(q - 1, 2 * q):
        exp[i] = exp[i - (q - 1)]
    return exp


def _poly_mul_gf2(a: int, b: int) -> int:
    out = 0
    while b:
        if b & 1:
            out ^= a
        a <<= 1
        b >>= 1
    return out


def _minimal_poly(m: int, e: int, exp) -> int:
    """Minimal polynomial over GF(2) of alpha^e, as an int (bit i = coeff of x^i)."""
    q1 = (1 << m) - 1
    conj = []
    x = e % q1
    while x not in conj:
        conj.append(x)
        x = (2 * x) % q1
    # product of (x - alpha^c) computed over GF(2^m); coefficients end up in GF(2)
    log = {exp[i]: i for i in range(q1)}

    def gmul(a, b):
        if a == 0 or b == 0:
            return 0
        return exp[(log[a] + log[b]) % q1]

    coeffs = [1]  # lowest degree first, elements of GF(2^m)
    for c in conj:
        root = exp[c]
        new = [0] * (len(coeffs) + 1)
        for i, a in enumerate(coeffs):
            new[i + 1] ^= a          # a * x
            new[i] ^= gmul(a, root)  # a * root  (minus == plus in char 2)
        coeffs = new
    out = 0
    for i, a in enumerate(coeffs):
        if a not in (0, 1):
            raise AssertionError("minimal polynomial not binary")
        out |= a << i
    return out


def _rank_rows(rows, ncols):
    """Row-reduce GF(2) rows (ints); return a list of independent rows."""
    basis = []  # list of (pivot_bit, row)
    for r in rows:
        for piv, b in basis:
            if (r >> piv) & 1:
                r ^= b
        if r:
            piv = r.bit_length() - 1
            basis.append((piv, r))
    return [b for _, b in basis]


def ebch(n: int, k: int) -> Code:
    """Extended BCH [n, k] code, n = 2^m, with the conventions in the module doc."""
    m = int(round(math.log2(n)))
    if 1 << m != n or m not in PRIM_POLY:
        raise ValueError(f"unsupported eBCH length {n}")
    nc = n - 1
    exp = _gf_tables(m)
    g = 1
    seen = set()
    t = 0
    while True:
        t += 1
        e = 2 * t - 1
        mp = _minimal_poly(m, e, exp)
        if mp not in seen:
            seen.add(mp)
            g = _poly_mul_gf2(g, mp)
        kc = nc - (g.bit_length() - 1)
        if kc <= k:
            break
    if kc != k:
        raise ValueError(f"no eBCH code [{n},{k}] (got k={kc} at t={t})")
    rc = nc - kc  # cyclic-code redundancy

    # systematic generator of the cyclic code, then the overall parity column
    G = np.zeros((k, n), dtype=np.uint8)
    for i in range(k):
        msg = 1 << (rc + i)          # x^rc * x^i
        rem = msg
        for d in range(nc - 1, rc - 1, -1):   # polynomial remainder mod g
            if (rem >> d) & 1:
                rem ^= g << (d - rc)
        cw = msg ^ rem
        for j in range(nc):
            G[i, j] = (cw >> j) & 1
        G[i, n - 1] = int(G[i, :nc].sum() & 1)
    info_pos = tuple(range(rc, rc + k))

    # parity-check rows: alpha^{(2i-1) j} bit planes for the distinct zeros, all-ones row
    rows = []
    for i in range(1, t + 1):
        e = 2 * i - 1
        for b in range(m):
            row = 0
            for j in range(nc):
                if (exp[(e * j) % nc] >> b) & 1:
                    row |= 1 << j
            rows.append(row)
    rows = _rank_rows(rows, nc)
    rows.append((1 << n) - 1)  # overall parity over all n positions
    if len(rows) != n - k:
        raise AssertionError("parity-check rank mismatch")
    hcols = []
    for j in range(n):
        c = 0
        for r, row in enumerate(rows):
            c |= ((row >> j) & 1) << r
        hcols.append(c)
    code = Code(f"eBCH[{n},{k}]", n, k, tuple(hcols), G, info_pos,
                bool(np.all(G.sum(axis=1) % 2 == 0)))
    _check_code(code)
    return code


def code_from_generator(name: str, G: np.ndarray, info_pos) -> Code:
    """Build a Code from any full-rank systematic generator (rows = codewords)."""
    G = np.asarray(G, dtype=np.uint8) & 1
    k, n = G.shape
    # null space of G over GF(2): H rows are a basis of {h : G h = 0}
    gi = [int("".join(str(b) for b in row[::-1]), 2) for row in G]
    basis = _rank_rows(gi, n)
    if len(basis) != k:
        raise ValueError("generator not full rank")
    # brute-force-free null space: solve with reduced row echelon form
    A = G.copy().astype(np.uint8)
    piv_cols = []
    row = 0
    for col in range(n):
        sel = [r for r in range(row, k) if A[r, col]]
        if not sel:
            continue
        A[[row, sel[0]]] = A[[sel[0], row]]
        for r in range(k):
            if r != row and A[r, col]:
                A[r] ^= A[row]
        piv_cols.append(col)
        row += 1
        if row == k:
            break
    free = [c for c in range(n) if c not in piv_cols]
    hrows = []
    for f in free:
        v = np.zeros(n, dtype=np.uint8)
        v[f] = 1
        for r, pc in enumerate(piv_cols):
            v[pc] = A[r, f]
        hrows.append(v)
    hcols = []
    for j in range(n):
        c = 0
        for r, v in enumerate(hrows):
            c |= int(v[j]) << r
        hcols.append(c)
    code = Code(name, n, k, tuple(hcols), G, tuple(int(p) for p in info_pos),
                bool(np.all(G.sum(axis=1) % 2 == 0)))
    _check_code(code)
    return code


def _check_code(code: Code) -> None:
    H = code.H()
    if np.any((code.G.astype(np.int64) @ H.T.astype(np.int64)) % 2):
        raise AssertionError(f"{code.name}: G H^T != 0")
    sub = code.G[:, list(code.info_pos)]
    if not np.array_equal(sub, np.eye(code.k, dtype=np.uint8)):
        raise AssertionError(f"{code.name}: generator not systematic on info_pos")


# Products of 0/1 matrices go through float32 BLAS: every sum is an integer of at
# most 128, exact in float32, and its parity is taken afterwards.
def _gf2_matmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return (np.matmul(a.astype(np.float32), b.astype(np.float32)).astype(np.int64) & 1).astype(np.uint8)


def encode(code: Code, info: np.ndarray) -> np.ndarray:
    """info (..., k) bits -> codewords (..., n) uint8."""
    return _gf2_matmul(np.asarray(info), code.G)


def encode_product(code: Code, info: np.ndarray) -> np.ndarray:
    """info (F, k, k) -> product codewords (F, n, n): k rows first, then n columns."""
    rows = _gf2_matmul(np.asarray(info), code.G)                 # (F, k, n)
    cols = _gf2_matmul(np.swapaxes(rows, -1, -2), code.G)        # (F, n, n): [col j][row i]
    return np.ascontiguousarray(np.swapaxes(cols, -1, -2))


# ----------------------------------------------------------------------------
# QC-GLDPC codes
# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Gldpc:
    """A QC-GLDPC code over a component code: G (dim, n*n) systematic on info_pos."""
    component: Code
    dim: int
    G: np.ndarray
    info_pos: tuple

    @property
    def n(self) -> int:
        return self.component.n


def _gldpc_checks(code: Code) -> np.ndarray:
    """(2n(n-k), n*n) parity-check matrix of the QC-GLDPC code over `code`."""
    n, r = code.n, code.r
    Hc = code.H()
    rows = []
    for block_row in range(2):
        for cn in range(n):
            # bit j of check node cn lies in block j, at column cn (first block row)
            # or at column (cn + j) mod n (second block row: the identity rotated by j)
            cols = [j * n + ((cn + (j if block_row else 0)) % n) for j in range(n)]
            for q in range(r):
                row = np.zeros(n * n, dtype=np.uint8)
                row[cols] = Hc[q]
                rows.append(row)
    return np.array(rows, dtype=np.uint8)


_GLDPC_CACHE: dict = {}


def gldpc(code: Code) -> Gldpc:
    """QC-GLDPC code with `code` as every component, and a systematic generator."""
    key = (code.name, code.n, code.k)
    if key in _GLDPC_CACHE:
        return _GLDPC_CACHE[key]
    H = _gldpc_checks(code)
    m, N = H.shape
    A = H.copy()
    piv = []
    row = 0
    for col in range(N):
        nz = np.nonzero(A[row:, col])[0]
        if nz.size == 0:
            continue
        p = row + nz[0]
        if p != row:
            A[[row, p]] = A[[p, row]]
        hit = np.nonzero(A[:, col])[0]
        hit = hit[hit != row]
        A[hit] ^= A[row]
        piv.append(col)
        row += 1
        if row == m:
            break
    free = [c for c in range(N) if c not in set(piv)]
    # one generator row per free column: 1 there, and the pivot columns that cancel it
    G = np.zeros((len(free), N), dtype=np.uint8)
    for i, f in enumerate(free):
        G[i, f] = 1
        for r_, pc in enumerate(piv):
            G[i, pc] = A[r_, f]
    if np.any(_gf2_matmul(G, H.T)):
        raise AssertionError("QC-GLDPC generator: G H^T != 0")
    g = Gldpc(code, len(free), G, tuple(free))
    _GLDPC_CACHE[key] = g
    return g


def gldpc_frames(g: Gldpc, ebn0_db, seed: int, frame_ids, batch: int = 4096):
    """QC-GLDPC frames over BPSK-AWGN at rate dim/n^2.  Returns (llr (F,n,n) float64,
    codewords (F,n,n) uint8, info (F,dim) uint8); element [j, c] is variable node j*n + c."""
    frame_ids = np.asarray(frame_ids, dtype=np.uint64)
    F = frame_ids.shape[0]
    n = g.n
    rate = g.dim / (n * n)
    eb = np.broadcast_to(np.asarray(ebn0_db, dtype=np.float64), (F,))
    llr = np.empty((F, n, n), dtype=np.float64)
    cw = np.empty((F, n, n), dtype=np.uint8)
    info = np.empty((F, g.dim), dtype=np.uint8)
    for s in range(0, F, batch):
        ids = frame_ids[s:s + batch]
        u = info_bits(seed, ids, g.dim)
        c = _gf2_matmul(u, g.G).reshape(-1, n, n)
        z = gaussians(seed, ids, n * n).reshape(-1, n, n)
        s2 = 1.0 / (2.0 * rate * 10.0 ** (eb[s:s + batch] / 10.0))
        x = 1.0 - 2.0 * c.astype(np.float64)
        r = x + np.sqrt(s2)[:, None, None] * z
        llr[s:s + batch] = 2.0 * r / s2[:, None, None]
        cw[s:s + batch] = c
        info[s:s + batch] = u
    return llr, cw, info


# ----------------------------------------------------------------------------
# counter-based random numbers
# ----------------------------------------------------------------------------
def _mix_int(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _mix_np(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(0xBF58476D1CE4E5B9)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _stream_keys(seed: int, frames: np.ndarray, stream: int) -> np.ndarray:
    k1 = _mix_int(seed ^ 0xA0761D6478BD642F)
    frames = np.asarray(frames, dtype=np.uint64)
    with np.errstate(over="ignore"):
        k2 = np.uint64(k1) ^ (frames * np.uint64(GAMMA)) ^ np.uint64((stream * 0xE7037ED1A0B428DB) & MASK64)
        return _mix_np(k2)


def splitmix_stream(seed: int, frames, stream: int, count: int) -> np.ndarray:
    """(len(frames), count) uint64: outputs 0..count-1 of each frame's stream."""
    keys = _stream_keys(seed, np.atleast_1d(frames), stream)
    with np.errstate(over="ignore"):
        ctr = (np.arange(1, count + 1, dtype=np.uint64) * np.uint64(GAMMA))
        return _mix_np(keys[:, None] + ctr[None, :])


def info_bits(seed: int, frames, count: int) -> np.ndarray:
    return (splitmix_stream(seed, frames, 0, count) >> np.uint64(63)).astype(np.uint8)


def gaussians(seed: int, frames, count: int, stream: int = 1) -> np.ndarray:
    npair = (count + 1) // 2
    o = splitmix_stream(seed, frames, stream, 2 * npair)
    u1 = ((o[:, 0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (o[:, 1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.empty((o.shape[0], 2 * npair), dtype=np.float64)
    z[:, 0::2] = rad * np.cos(2.0 * np.pi * u2)
    z[:, 1::2] = rad * np.sin(2.0 * np.pi * u2)
    return z[:, :count]


def rician_qpsk_llr(cw: np.ndarray, ebn0_db, rate: float, K: float, nc: int, seed: int, frame_ids) -> np.ndarray:
    """Channel LLRs (F, N) float64 of codewords cw (F, N) sent over block Rician fading with QPSK
    (module docstring); N = 2 t nc."""
    cw = np.asarray(cw, dtype=np.uint8)
    F, N = cw.shape
    if N % (2 * nc):
        raise ValueError("N must be a multiple of 2 * nc")
    ids = np.asarray(frame_ids, dtype=np.uint64)
    nsym, t = N // 2, N // (2 * nc)
    eb = np.broadcast_to(np.asarray(ebn0_db, dtype=np.float64), (F,))
    s2 = 1.0 / (2.0 * rate * 10.0 ** (eb / 10.0))                              # Delta = 1
    perm = np.argsort(splitmix_stream(seed, ids, 3, N), axis=1, kind="stable")  # interleaved bit i = code bit perm[i]
    b = np.take_along_axis(cw, perm, axis=1)
    x = (1.0 - 2.0 * b[:, 0::2]) + 1j * (1.0 - 2.0 * b[:, 1::2])
    g = gaussians(seed, ids, 2 * t, stream=2)
    h_ra = np.sqrt(0.5) * (g[:, 0::2] + 1j * g[:, 1::2])
    h = np.sqrt(K / (K + 1.0)) + np.sqrt(1.0 / (K + 1.0)) * h_ra              # (F, t)
    hs = np.repeat(h, nc, axis=1)                                               # (F, nsym)
    z = gaussians(seed, ids, 2 * nsym, stream=1)
    noise = np.sqrt(s2)[:, None] * (z[:, 0::2] + 1j * z[:, 1::2])
    y = hs * x + noise
    yh = y * np.conj(hs)
    li = np.empty((F, N), dtype=np.float64)
    li[:, 0::2] = 2.0 * yh.real / s2[:, None]
    li[:, 1::2] = 2.0 * yh.imag / s2[:, None]
    llr = np.empty_like(li)
    np.put_along_axis(llr, perm, li, axis=1)
    return llr


def rician_product_frames(code: Code, ebn0_db, K: float, nc: int, seed: int, frame_ids, batch: int = 4096):
    """Product-code frames over block Rician fading with QPSK.  Returns (llr (F,n,n), codewords
    (F,n,n) uint8, info (F,k,k) uint8)."""
    frame_ids = np.asarray(frame_ids, dtype=np.uint64)
    F = frame_ids.shape[0]
    n, k = code.n, code.k
    eb = np.broadcast_to(np.asarray(ebn0_db, dtype=np.float64), (F,))
    llr = np.empty((F, n, n), dtype=np.float64)
    cw = np.empty((F, n, n), dtype=np.uint8)
    info = np.empty((F, k, k), dtype=np.uint8)
    for s in range(0, F, batch):
        ids = frame_ids[s:s + batch]
        u = info_bits(seed, ids, k * k).reshape(-1, k, k)
        c = encode_product(code, u)
        llr[s:s + batch] = rician_qpsk_llr(c.reshape(len(ids), -1), eb[s:s + batch], (k * k) / (n * n), K, nc,
                                           seed, ids).reshape(-1, n, n)
        cw[s:s + batch] = c
        info[s:s + batch] = u
    return llr, cw, info


def sigma2(ebn0_db: float, rate: float) -> float:
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def bpsk_awgn_llr(codewords: np.ndarray, noise: np.ndarray, s2: float) -> np.ndarray:
    x = 1.0 - 2.0 * codewords.astype(np.float64)
    r = x + math.sqrt(s2) * noise
    return 2.0 * r / s2


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def product_frames(code: Code, ebn0_db, seed: int, frame_ids, batch: int = 4096):
    """Product-code frames over BPSK-AWGN.

    ebn0_db is a scalar or one value per frame.  Returns (llr (F,n,n) float64,
    codewords (F,n,n) uint8, info (F,k,k) uint8).
    """
    frame_ids = np.asarray(frame_ids, dtype=np.uint64)
    F = frame_ids.shape[0]
    n, k = code.n, code.k
    rate = (k * k) / (n * n)
    eb = np.broadcast_to(np.asarray(ebn0_db, dtype=np.float64), (F,))
    llr = np.empty((F, n, n), dtype=np.float64)
    cw = np.empty((F, n, n), dtype=np.uint8)
    info = np.empty((F, k, k), dtype=np.uint8)
    for s in range(0, F, batch):
        ids = frame_ids[s:s + batch]
        u = info_bits(seed, ids, k * k).reshape(-1, k, k)
        c = encode_product(code, u)
        z = gaussians(seed, ids, n * n).reshape(-1, n, n)
        s2 = 1.0 / (2.0 * rate * 10.0 ** (eb[s:s + batch] / 10.0))
        x = 1.0 - 2.0 * c.astype(np.float64)
        r = x + np.sqrt(s2)[:, None, None] * z
        llr[s:s + batch] = 2.0 * r / s2[:, None, None]
        cw[s:s + batch] = c
        info[s:s + batch] = u
    return llr, cw, info


def component_words(code: Code, ebn0_db, seed: int, word_ids, batch: int = 1 << 16):
    """Independent component words over BPSK-AWGN at rate k/n.

    Returns (llr (W,n) float64, codewords (W,n) uint8, info (W,k) uint8).
    """
    word_ids = np.asarray(word_ids, dtype=np.uint64)
    Wn = word_ids.shape[0]
    n, k = code.n, code.k
    rate = k / n
    eb = np.broadcast_to(np.asarray(ebn0_db, dtype=np.float64), (Wn,))
    llr = np.empty((Wn, n), dtype=np.float64)
    cw = np.empty((Wn, n), dtype=np.uint8)
    info = np.empty((Wn, k), dtype=np.uint8)
    for s in range(0, Wn, batch):
        ids = word_ids[s:s + batch]
        u = info_bits(seed, ids, k)
        c = encode(code, u)
        z = gaussians(seed, ids, n)
        s2 = 1.0 / (2.0 * rate * 10.0 ** (eb[s:s + batch] / 10.0))
        x = 1.0 - 2.0 * c.astype(np.float64)
        r = x + np.sqrt(s2)[:, None] * z
        llr[s:s + batch] = 2.0 * r / s2[:, None]
        cw[s:s + batch] = c
        info[s:s + batch] = u
    return llr, cw, info


def mixed_product_frames(codes, ebn0_lo: float, ebn0_hi: float, seed: int, frame_ids):
    """Product frames whose code and Eb/N0 are drawn per frame.

    Frame f takes code index floor(u0 * len(codes)) and Eb/N0 = lo + (hi - lo) u1,
    with (u0, u1) the first two outputs of stream 2 of (seed, f) mapped to [0, 1)
    by (o >> 11) 2^-53; its bits and noise are those of product_frames(code, ...,
    seed, [f]).  Returns (code_idx (F,) uint8, ebn0 (F,), offsets (F,) int64,
    llr flat float64, codewords flat uint8), frames packed row-major one after the
    other.
    """
    frame_ids = np.asarray(frame_ids, dtype=np.uint64)
    F = frame_ids.shape[0]
    u = (splitmix_stream(seed, frame_ids, 2, 2) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    cidx = np.minimum((u[:, 0] * len(codes)).astype(np.int64), len(codes) - 1).astype(np.uint8)
    ebn0 = ebn0_lo + (ebn0_hi - ebn0_lo) * u[:, 1]
    sizes = np.array([codes[c].n ** 2 for c in cidx], dtype=np.int64)
    offsets = np.zeros(F, dtype=np.int64)
    if F:
        offsets[1:] = np.cumsum(sizes)[:-1]
    total = int(sizes.sum())
    llr = np.empty(total, dtype=np.float64)
    cw = np.empty(total, dtype=np.uint8)
    for c, code in enumerate(codes):
        sel = np.nonzero(cidx == c)[0]
        if sel.size == 0:
            continue
        l, w, _ = product_frames(code, ebn0[sel], seed, frame_ids[sel])
        nn = code.n * code.n
        idx = offsets[sel][:, None] + np.arange(nn)[None, :]
        llr[idx] = l.reshape(-1, nn)
        cw[idx] = w.reshape(-1, nn)
    return cidx, ebn0, offsets, llr, cw
