"""Pins for the oracle's quadtree (adaptive range) encoder: the two limits
of the tolerance reduce it to the plain search at the largest and at the
smallest range size, the leaves tile the image once, every split and every
kept leaf obeys the rule, planted exact ranges are kept whole, and every
level's codes agree with the independent brute-force search."""
import numpy as np
import pytest

from oracle import oracle as O
from fic_inputs import gen_image
from brute import brute_encode
from planted import planted_image, PLANTS_64_N8

FIELDS = ("domain", "iso", "s_idx", "o_idx", "err")


def zorder_positions(H, W, n_max, n_min):
    """(y, x) of the n_min ranges in the leaf order of a fully split tree."""
    out = []

    def walk(y, x, n):
        if n == n_min:
            out.append((y, x))
            return
        h = n // 2
        for dy, dx in ((0, 0), (0, h), (h, 0), (h, h)):
            walk(y + dy, x + dx, h)

    for ry in range(H // n_max):
        for rx in range(W // n_max):
            walk(ry * n_max, rx * n_max, n_max)
    return out


@pytest.mark.parametrize("n_max,n_min,step", [(8, 4, 4), (16, 4, 4), (16, 8, 8)])
def test_infinite_tolerance_is_the_plain_search_at_the_largest_size(n_max, n_min, step):
    img = gen_image(64, 64, 8, 41)
    q = O.encode_quadtree(img, n_max, n_min, step, np.inf)
    ref = O.encode(img, n_max, step)
    for k in FIELDS:
        np.testing.assert_array_equal(q[k], ref[k])
    assert np.all(q["size"] == n_max) and all(s.sum() == 0 for s in q["split"])


@pytest.mark.parametrize("n_max,n_min,step", [(8, 4, 4), (16, 4, 4)])
def test_negative_tolerance_is_the_plain_search_at_the_smallest_size(n_max, n_min, step):
    H = W = 64
    img = gen_image(H, W, 8, 42)
    q = O.encode_quadtree(img, n_max, n_min, step, -1.0)
    ref = O.encode(img, n_min, step)
    pos = zorder_positions(H, W, n_max, n_min)
    order = np.array([(y // n_min) * (W // n_min) + x // n_min for (y, x) in pos])
    for k in FIELDS:
        np.testing.assert_array_equal(q[k], ref[k][order])
    np.testing.assert_array_equal(q["y"], [p[0] for p in pos])
    np.testing.assert_array_equal(q["x"], [p[1] for p in pos])


@pytest.mark.parametrize("tau", [0.0, 4.0, 20.0, 80.0])
def test_leaves_tile_the_image_and_obey_the_split_rule(tau):
    H, W, n_max, n_min, step = 64, 48, 16, 4, 4
    img = gen_image(H, W, 8, 43)
    q = O.encode_quadtree(img, n_max, n_min, step, tau)
    cover = np.zeros((H, W), np.int32)
    for y, x, n in zip(q["y"], q["x"], q["size"]):
        cover[y:y + n, x:x + n] += 1
    assert np.all(cover == 1)
    # a leaf above the smallest size was kept: residual within tolerance
    for n, e in zip(q["size"], q["err"]):
        if n > n_min:
            assert e <= tau * n * n
    # a split range exceeded it (its code at that size, from the plain search)
    for lvl, flags in enumerate(q["split"]):
        n = n_max >> lvl
        idx = np.nonzero(flags)[0]
        if len(idx):
            c = O.encode_ranges(img, n, step, idx)
            assert np.all(c["err"] > tau * n * n)


def test_planted_exact_ranges_are_kept_whole():
    H = W = 64
    n, step = 8, 4
    img = planted_image(H, W, n, step, 8, 23, PLANTS_64_N8)
    q = O.encode_quadtree(img, n, 4, step, 0.0)
    planted = {r for (r, *_rest) in PLANTS_64_N8}
    nx = W // n
    for r in planted:
        assert q["split"][0][r] == 0
    kept = {(int(y), int(x)) for y, x, s in zip(q["y"], q["x"], q["size"]) if s == n}
    assert {((r // nx) * n, (r % nx) * n) for r in planted} <= kept


@pytest.mark.parametrize("n_max,n_min,step,tau", [(8, 4, 4, 10.0), (16, 4, 8, 30.0)])
def test_every_level_matches_brute_force(n_max, n_min, step, tau):
    H = W = 48 if n_max == 8 else 64
    img = gen_image(H, W, 8, 44)
    q = O.encode_quadtree(img, n_max, n_min, step, tau)
    by_size = {}
    n = n_max
    while n >= n_min:
        by_size[n] = brute_encode(img, n, step)
        n //= 2
    for i in range(len(q["y"])):
        y, x, n = int(q["y"][i]), int(q["x"][i]), int(q["size"][i])
        r = (y // n) * (W // n) + x // n
        for k in FIELDS:
            assert q[k][i] == by_size[n][k][r], (i, k)
