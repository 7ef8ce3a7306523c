"""Pins for the oracle's full search (Alg. 2 / Alg. 3): brute force on tiny
images, planted self-similar images, transpose invariance, and the flat
("shadow") range rule."""
import numpy as np
import pytest

from oracle import oracle as O
from fic_inputs import gen_image
from brute import brute_encode
from planted import planted_image, PLANTS_64_N8

KEYS = ("domain", "iso", "s_idx", "o_idx", "err")


def _same(a, b):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("H,W,n,step,bits,seed", [
    (16, 16, 4, 4, 8, 0), (16, 16, 4, 2, 8, 1), (24, 16, 4, 4, 8, 2), (16, 24, 4, 3, 8, 3),
    (16, 16, 2, 1, 8, 4), (32, 32, 4, 4, 8, 5), (16, 16, 4, 2, 12, 6), (32, 32, 8, 4, 8, 7),
    (32, 32, 8, 8, 12, 8), (24, 24, 4, 4, 12, 9),
])
def test_oracle_matches_brute_force(H, W, n, step, bits, seed):
    rng = np.random.default_rng(seed)
    P = 1 << bits
    kind = seed % 3
    if kind == 0:
        img = rng.integers(0, P, size=(H, W))
    elif kind == 1:
        img = gen_image(H, W, bits, seed)
    else:   # few levels -> many exact ties between candidates
        img = rng.integers(0, 3, size=(H, W)) * (P // 4)
    img = np.asarray(img, np.uint16)
    _same(O.encode(img, n, step, bits=bits), brute_encode(img, n, step, bits=bits))


@pytest.mark.parametrize("bits", [8, 12])
def test_planted_codes_recovered(bits):
    H = W = 32
    n, step = 4, 4
    P = 1 << bits
    plants = [(63, (0, 0), 1, 0.5, 8.0 * (P // 256)),     # range (7,7), domain at (0,0)
              (56, (0, 5), 4, -0.5, P / 2.0),             # range (7,0), domain at (0,20)
              (7, (5, 0), 6, 0.75, 0.0),                  # range (0,7), domain at (20,0)
              (35, (1, 1), 3, 0.25, P / 4.0)]             # range (4,3), domain at (4,4)
    img = planted_image(H, W, n, step, bits, 17 + bits, plants)
    ora = O.encode(img, n, step, bits=bits)
    bru = brute_encode(img, n, step, bits=bits)
    _same(ora, bru)
    nx = (W - 2 * n) // step + 1
    dlt = 2 * P // 128
    for (r, (dy, dx), k, s, o) in plants:
        assert ora["err"][r] == 0.0
        assert ora["domain"][r] == dy * nx + dx and ora["iso"][r] == k
        assert ora["s_idx"][r] == int((s + 1) * 16) and ora["o_idx"][r] == int((o + P) / dlt)


def test_planted_codes_n8():
    img = planted_image(64, 64, 8, 4, 8, 23, PLANTS_64_N8)
    ora = O.encode(img, 8, 4)
    for (r, (dy, dx), k, s, o) in PLANTS_64_N8:
        assert ora["err"][r] == 0.0
        assert ora["domain"][r] == dy * 13 + dx and ora["iso"][r] == k
        assert ora["s_idx"][r] == int((s + 1) * 16) and ora["o_idx"][r] == int((o + 256) / 4)


@pytest.mark.parametrize("bits,n,step", [(8, 4, 4), (8, 4, 2), (12, 4, 4)])
def test_min_error_invariant_under_transpose(bits, n, step):
    # the transform set is closed under transposition and the grid is symmetric,
    # so range (y, x) of I and range (x, y) of I^T have the same minimum residual
    img = gen_image(48, 48, bits, 21)
    a = O.encode(img, n, step, bits=bits)
    b = O.encode(np.ascontiguousarray(img.T), n, step, bits=bits)
    g = 48 // n
    ea = a["err"].reshape(g, g)
    eb = b["err"].reshape(g, g)
    np.testing.assert_array_equal(ea, eb.T)


def test_flat_ranges_take_first_candidate():
    # a range with no variance fits every candidate with s = 0 and the same
    # offset, so every candidate ties and the first one (d = 0, k = 0) is kept
    img = gen_image(64, 64, 8, 1)
    out = O.encode(img, 4, 4)
    b = img.reshape(16, 4, 16, 4).transpose(0, 2, 1, 3).reshape(256, 16).astype(np.float64)
    flat = b.std(1) == 0
    assert flat.sum() > 50
    assert np.all(out["domain"][flat] == 0) and np.all(out["iso"][flat] == 0)
    assert np.all(out["s_idx"][flat] == 16)
    mean = b[flat].mean(1)
    np.testing.assert_array_equal(out["o_idx"][flat], np.floor((mean + 256) / 4 + 0.5))


def test_range_subset_equals_full():
    img = gen_image(64, 64, 8, 1)
    full = O.encode(img, 4, 4)
    part = O.encode(img, 4, 4, r_begin=100, r_end=140)
    for k in KEYS:
        np.testing.assert_array_equal(full[k][100:140], part[k])


def test_range_list_equals_full():
    img = gen_image(64, 64, 8, 1)
    full = O.encode(img, 4, 4)
    rs = np.array([255, 0, 17, 17, 128])
    part = O.encode_ranges(img, 4, 4, rs)
    for k in KEYS:
        np.testing.assert_array_equal(full[k][rs], part[k])


def test_invalid_parameters_rejected():
    img = np.zeros((16, 16), np.uint16)
    for args in [dict(n=3, step=4), dict(n=4, step=0), dict(n=16, step=1)]:
        with pytest.raises(ValueError):
            O.encode(img, **args)
