"""Planted self-similar test images (test-side input construction).

A domain whose 2x2 cells are constant integers v has contracted values
exactly v.  Writing a range as b = s * T(v) + o, with T one of the eight
transforms (NumPy's rot90/fliplr) and (s, o) on the quantisation grid, makes
that candidate fit with zero residual (eq. 8).
"""
import numpy as np

from brute import transforms


# 64x64 image, 8x8 ranges, 16x16 domains at stride 4: four plants whose
# domains avoid every planted range.
PLANTS_64_N8 = [(63, (0, 0), 1, 0.5, 8.0), (56, (0, 6), 4, -0.5, 128.0),
                (39, (6, 0), 6, 0.75, 0.0), (35, (2, 2), 3, 0.25, 64.0)]


def planted_image(H, W, n, step, bits, seed, plants):
    """plants: list of (range_index, (dy, dx), k, s, o).  Domains must not
    overlap any planted range.  Returns the image (uint16)."""
    rng = np.random.default_rng(seed)
    P = 1 << bits
    img = rng.integers(0, P, size=(H, W)).astype(np.int64)
    for (r, (dy, dx), k, s, o) in plants:
        Y, X = dy * step, dx * step
        # random cell values, multiples of 4 so that s * v stays integral
        vals = 4 * rng.integers(1, P // 8, size=(n, n))
        img[Y:Y + 2 * n, X:X + 2 * n] = np.kron(vals, np.ones((2, 2), np.int64))
    for (r, _d, _k, _s, _o) in plants:
        ry, rx = divmod(r, W // n)
        for (_r, (dy, dx), _k2, _s2, _o2) in plants:
            Y, X = dy * step, dx * step
            assert not (ry * n < Y + 2 * n and Y < (ry + 1) * n and
                        rx * n < X + 2 * n and X < (rx + 1) * n), "range overlaps a planted domain"
    for (r, (dy, dx), k, s, o) in plants:
        Y, X = dy * step, dx * step
        vals = img[Y:Y + 2 * n:2, X:X + 2 * n:2]
        b = s * transforms(vals)[k].astype(np.float64) + o
        assert np.all(b == np.floor(b)) and b.min() >= 0 and b.max() <= P - 1, "plant off range"
        ry, rx = divmod(r, W // n)
        img[ry * n:(ry + 1) * n, rx * n:(rx + 1) * n] = b.astype(np.int64)
    return img.astype(np.uint16)
