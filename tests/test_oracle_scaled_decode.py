"""Pins for the oracle's decoder at another resolution (the code decoded at
z = 1/2, 2, 4 times the size it was encoded at): closed forms at every scale,
the fixed point of the scaled map against an independently built matrix,
and the averaging identity that ties every scale to the pinned 1x decoder.

Averaging identity: write D_z for the z x z block mean.  The transforms map
the 2x2 pixel group (2i, 2j) of a 2m-pixel block onto the group 2 sigma(i, j)
of the m-pixel block's transform, and a 2x2 mean of 2x2 cell means is the 4x4
mean, so D_2 applied after one step of the 2x map equals one step of the 1x
map applied after D_2.  From a constant start every iterate then satisfies
D_2(x_t at 2z) = x_t at z.  A scaled map with a wrong transform size, a
domain grid left unscaled or a mis-scaled range fails it."""
import numpy as np
import pytest

from oracle import oracle as O
from fic_inputs import gen_image
from test_oracle_decode import map_matrix, random_codes, range_const


def pool(x, z):
    """Mean over z x z blocks of the last two axes."""
    *lead, h, w = x.shape
    return x.reshape(*lead, h // z, z, w // z, z).mean(axis=(-3, -1))


SCALES = [(1, 2), (2, 1), (4, 1)]


@pytest.mark.parametrize("num,den", SCALES)
def test_zero_contrast_gives_offset_blocks(num, den):
    H = W = 32; n = 4; step = 4
    dom, iso, s, o = random_codes(H, W, n, step, 20)
    s[:] = 0.0
    traj = O.decode_scaled(H, W, n, step, num, den, dom, iso, s, o, 4, 128.0)
    nz = n * num // den
    assert traj.shape == (5, H * num // den, W * num // den)
    for t in range(1, 5):
        np.testing.assert_array_equal(traj[t], range_const(H * num // den, W * num // den, nz, o))


@pytest.mark.parametrize("num,den", SCALES)
def test_half_contrast_constant_offset_closed_form(num, den):
    H = W = 32; n = 8; step = 2
    dom, iso, s, o = random_codes(H, W, n, step, 21)
    s[:] = 0.5
    o[:] = -12.0
    traj = O.decode_scaled(H, W, n, step, num, den, dom, iso, s, o, 12, 128.0)
    for t in range(13):
        np.testing.assert_array_equal(traj[t], np.full(traj.shape[1:], -24.0 + (128.0 + 24.0) / 2 ** t))


def test_unit_scale_is_the_decoder():
    H, W, n, step = 32, 48, 4, 2
    dom, iso, s, o = random_codes(H, W, n, step, 22)
    np.testing.assert_array_equal(O.decode_scaled(H, W, n, step, 1, 1, dom, iso, s, o, 6, 128.0),
                                  O.decode(H, W, n, step, dom, iso, s, o, 6, 128.0))
    np.testing.assert_array_equal(O.decode_scaled(H, W, n, step, 3, 3, dom, iso, s, o, 6, 128.0),
                                  O.decode(H, W, n, step, dom, iso, s, o, 6, 128.0))


@pytest.mark.parametrize("H,W,n,step,seed", [(32, 48, 4, 2, 23), (64, 64, 8, 4, 24), (48, 32, 4, 4, 25)])
def test_averaging_ties_every_scale_to_the_unit_decode(H, W, n, step, seed):
    dom, iso, s, o = random_codes(H, W, n, step, seed, smax=1.0)
    T = 12
    x1 = O.decode(H, W, n, step, dom, iso, s, o, T, 128.0)
    for z in (2, 4):
        xz = O.decode_scaled(H, W, n, step, z, 1, dom, iso, s, o, T, 128.0)
        np.testing.assert_allclose(pool(xz, z), x1, rtol=0, atol=1e-9)
    xh = O.decode_scaled(H, W, n, step, 1, 2, dom, iso, s, o, T, 128.0)
    np.testing.assert_allclose(pool(x1, 2), xh, rtol=0, atol=1e-9)


def test_averaging_identity_on_encoded_codes():
    # the codes of a real (synthetic) slice, as the encoder produced them
    H = W = 64; n = 4; step = 4
    img = gen_image(H, W, 8, 26)
    c = O.encode(img, n, step)
    s, o = O.dequantize(c["s_idx"], c["o_idx"])
    x1 = O.decode(H, W, n, step, c["domain"], c["iso"], s, o, 12, 128.0)
    x4 = O.decode_scaled(H, W, n, step, 4, 1, c["domain"], c["iso"], s, o, 12, 128.0)
    np.testing.assert_allclose(pool(x4, 4), x1, rtol=0, atol=1e-9)


def test_scaled_map_fixed_point_against_independent_matrix():
    # at 2x the map is the same construction on the scaled grid: its dense
    # matrix (built by NumPy's transforms of an index grid) fixes the limit
    H, W, n, step = 16, 24, 4, 2
    dom, iso, s, o = random_codes(H, W, n, step, 27)
    Hz, Wz, nz, sz = 2 * H, 2 * W, 2 * n, 2 * step
    M = map_matrix(Hz, Wz, nz, sz, dom, iso, s)
    ovec = range_const(Hz, Wz, nz, o).ravel()
    xstar = np.linalg.solve(np.eye(Hz * Wz) - M, ovec)
    traj = O.decode_scaled(H, W, n, step, 2, 1, dom, iso, s, o, 12, 128.0)
    for t in range(12):
        np.testing.assert_allclose(traj[t + 1].ravel(), M @ traj[t].ravel() + ovec, rtol=0, atol=1e-9)
    c = np.abs(s).max()
    assert np.abs(traj[-1].ravel() - xstar).max() <= c ** 12 * np.abs(128.0 - xstar).max() * (1 + 1e-12) + 1e-9


@pytest.mark.parametrize("num,den,n,step", [(1, 3, 4, 4), (1, 2, 4, 3), (1, 8, 4, 4), (0, 1, 4, 4),
                                            (3, 2, 4, 3), (8, 1, 8, 4)])
def test_scale_must_keep_whole_pixels(num, den, n, step):
    H = W = 48
    dom, iso, s, o = random_codes(H, W, n, step, 28)
    with pytest.raises(ValueError):
        O.decode_scaled(H, W, n, step, num, den, dom, iso, s, o, 2, 128.0)
