"""Pins for the oracle's least squares, quantisation and residual
(eqs. 8-12): closed forms, special cases and exact rational arithmetic."""
from fractions import Fraction
import math

import numpy as np
import pytest

from oracle import oracle as O


def frac_fit(a4, b, bits, s_bits, o_bits):
    """Exact-rational reference of one fit; a4 are integer cell sums (4 a)."""
    K = len(b)
    a = [Fraction(int(x), 4) for x in a4]
    b = [Fraction(int(x)) for x in b]
    ma = sum(a) / K
    mb = sum(b) / K
    var = sum((x - ma) ** 2 for x in a)
    cov = sum((x - ma) * (y - mb) for x, y in zip(a, b))
    s = Fraction(0) if var == 0 else cov / var
    S = 2 ** (s_bits - 1)
    j = min(max(math.floor((s + 1) * S + Fraction(1, 2)), 0), 2 * S - 1)
    sq = Fraction(j, S) - 1
    o = mb - sq * ma
    P = 2 ** bits
    dlt = Fraction(2 * P, 2 ** o_bits)
    m = min(max(math.floor((o + P) / dlt + Fraction(1, 2)), 0), 2 ** o_bits - 1)
    oq = m * dlt - P
    E = sum((sq * x + oq - y) ** 2 for x, y in zip(a, b))
    return j, m, sq, oq, E


@pytest.mark.parametrize("bits,n", [(8, 4), (8, 8), (12, 4), (12, 8)])
def test_fit_exact_vs_fractions(bits, n):
    rng = np.random.default_rng(100 + bits + n)
    K = n * n
    P = 2 ** bits
    cases = []
    for t in range(300):
        a4 = rng.integers(0, 4 * (P - 1) + 1, size=K)
        b = rng.integers(0, P, size=K)
        if t % 5 == 1:      # correlated
            b = np.clip(np.rint(a4 / 4 * rng.uniform(-1, 1) + rng.uniform(0, P)), 0, P - 1).astype(int)
        if t % 7 == 2:      # saturated
            a4 = np.full(K, 4 * (P - 1)); a4[rng.integers(0, K)] = rng.integers(0, 4 * P - 3)
            b = np.full(K, P - 1)
        if t % 11 == 3:     # flat domain
            a4 = np.full(K, rng.integers(0, 4 * P - 3))
        cases.append((a4, b))
    for a4, b in cases:
        j, m, s, o, e = O.fit(a4 / 4.0, b, bits=bits)
        fj, fm, fs, fo, fe = frac_fit(a4, b, bits, 5, 7)
        assert (j, m) == (fj, fm)
        assert Fraction(s) == fs and Fraction(o) == fo
        assert Fraction(e) == fe        # residual is exact in double


def test_planted_linear_block_recovered():
    # b = s a + o with (s, o) on the grid and a non-constant -> s*, o* exact, E = 0
    rng = np.random.default_rng(3)
    for bits in (8, 12):
        P = 2 ** bits
        for s_val in (-1.0, -0.5, -0.25, 0.25, 0.5, 0.75, 0.9375):
            for _ in range(5):
                v = rng.integers(0, P // 2, size=16).astype(np.float64)  # integer a
                dlt = 2 * P / 128
                lo = math.ceil(max(0.0, -(s_val * v).min()) / dlt)
                hi = math.floor((P - 1 - max(0.0, (s_val * v).max())) / dlt)
                o_val = dlt * rng.integers(lo, hi + 1)
                b = s_val * v + o_val
                if not np.all(b == np.floor(b)):
                    continue
                j, m, s, o, e = O.fit(v, b, bits=bits)
                assert s == s_val and o == o_val and e == 0.0
                assert j == int((s_val + 1) * 16) and m == int((o_val + P) / dlt)


def test_flat_domain_uses_eqs_11_12():
    b = np.arange(16, dtype=np.float64) * 3
    a = np.full(16, 17.25)
    j, m, s, o, e = O.fit(a, b)
    assert s == 0.0 and j == 16                    # eq. (11)
    mean = b.mean()                                # eq. (12) then quantised
    assert o == 4 * math.floor(mean / 4 + 0.5)
    assert e == float(((o - b) ** 2).sum())


def test_flat_range():
    a = np.random.default_rng(0).integers(0, 1021, 16) / 4.0
    b = np.full(16, 101.0)
    j, m, s, o, e = O.fit(a, b)
    assert s == 0.0 and o == 100.0 and e == 16.0   # q(101) = 100 on the step-4 grid


def test_quantiser_grid_points_midpoints_and_clamps():
    # contrast exactly on grid points and exactly on midpoints (round half up)
    a = np.array([0, 4, 0, 4] * 4, dtype=np.float64)       # a in {0, 4}, mean 2
    for num in range(-40, 40):
        s_true = num / 32.0                                 # grid points and midpoints
        b = s_true * a + 128.0
        j, m, s, o, e = O.fit(a, b)
        expect = min(max(math.floor((s_true + 1) * 16 + 0.5), 0), 31)
        assert j == expect
    # clamps: very steep positive and negative slopes
    a = np.array([0.0, 1.0] * 8)
    b = np.array([0.0, 255.0] * 8)
    assert O.fit(a, b)[0] == 31
    assert O.fit(a, b[::-1].copy())[0] == 0
    # offset clamp at the top of [-P, P - delta_o]: b = 255 - a gives s* = -1 and
    # o* = 255, which rounds to index 128 and is clamped to 127 (o_q = 252)
    a = np.array([0.0, 255.0] * 8)
    b = np.array([255.0, 0.0] * 8)
    assert O.fit(a, b) == (0, 127, -1.0, 252.0, 16 * 3.0 ** 2)
    # contrast clamp at the top: s* = 1 -> index 32 clamped to 31 (s_q = 15/16)
    a = np.full(16, 255.0); a[0] = 0.0
    b = a.copy()
    j, m, s, o, e = O.fit(a, b)
    fj, fm, fs, fo, fe = frac_fit((4 * a).astype(int), b.astype(int), 8, 5, 7)
    assert (j, m, s, o, e) == (31, fm, 15 / 16, float(fo), float(fe))


def test_residual_is_eq8_with_quantised_values():
    rng = np.random.default_rng(11)
    for _ in range(50):
        a = rng.integers(0, 1021, 64) / 4.0
        b = rng.integers(0, 256, 64).astype(np.float64)
        j, m, s, o, e = O.fit(a, b)
        assert s == j / 16 - 1 and o == m * 4 - 256
        assert e == float(((s * a + o - b) ** 2).sum())
