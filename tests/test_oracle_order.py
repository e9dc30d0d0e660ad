"""Pins for the oracle's ORBGRAND query order.

The order (basic ORBGRAND, cited in the paper's section on GRAND background):
patterns are sets of reliability ranks, queried by logistic weight W = sum of
ranks, then Hamming weight, then the rank tuple in lexicographic order; even
codes query only one weight parity.  Pinned here by brute force over all 2^n
subsets and by the generating function prod_i (1 + y x^i).
"""
import itertools

import numpy as np
import pytest

import oracle


def brute_order(n, parity):
    pats = []
    for w in range(n + 1):
        if parity >= 0 and w % 2 != parity:
            continue
        pats.extend(itertools.combinations(range(1, n + 1), w))
    return sorted(pats, key=lambda u: (sum(u), len(u), u))


@pytest.mark.parametrize("n", [1, 2, 5, 8, 11])
@pytest.mark.parametrize("parity", [0, 1, -1])
def test_order_equals_bruteforce_sort(n, parity):
    ref = brute_order(n, parity)
    got = oracle.order(n, parity, 1 << n)
    assert got == ref


def test_order_n16_odd_class_and_prefix():
    ref = brute_order(16, 1)
    assert len(ref) == 1 << 15
    assert oracle.order(16, 1, 1 << 15) == ref
    assert oracle.order(16, 1, 1000) == ref[:1000]


def _gf_counts(n, wmax_sum):
    # coefficient table c[W][parity] of prod_{i=1}^n (1 + y x^i), y^2 = 1 tracked as parity
    c = np.zeros((wmax_sum + 1, 2), dtype=object)
    c[0, 0] = 1
    for i in range(1, n + 1):
        nc = c.copy()
        for W in range(i, wmax_sum + 1):
            nc[W, 0] += c[W - i, 1]
            nc[W, 1] += c[W - i, 0]
        c = nc
    return c


def test_order_counts_match_generating_function_n8():
    c = _gf_counts(8, 36)
    # distinct-part partitions with parts <= 8: 1,1,1,2,2,3,4,5,6,7,8,...; total 256
    tot = [int(c[W, 0] + c[W, 1]) for W in range(37)]
    assert tot[:12] == [1, 1, 1, 2, 2, 3, 4, 5, 6, 7, 8, 9]
    assert sum(tot) == 256
    pats = oracle.order(8, -1, 256)
    hist = np.bincount([sum(u) for u in pats], minlength=37)
    assert list(hist) == tot


@pytest.mark.parametrize("n,parity", [(32, 0), (64, 1), (128, 0), (128, 1)])
def test_order_counts_match_generating_function_large(n, parity):
    Wcut = 30
    c = _gf_counts(n, Wcut)
    want = [int(c[W, parity]) for W in range(Wcut + 1)]
    total = sum(want)
    pats = oracle.order(n, parity, total + 5)
    hist = np.bincount([sum(u) for u in pats[:total]], minlength=Wcut + 1)
    assert list(hist[:Wcut + 1]) == want
    assert sum(pats[total]) == Wcut + 1          # the next pattern starts the next weight
    ws = [len(u) for u in pats]
    assert all(w % 2 == parity for w in ws)
