"""Planted self-similar test images (test-side input construction).

A domain whose 2x2 cells are constant integers v has contracted values
exactly v.  Writing a range as b = s * T(v) + o, with T one of the eight
transforms (NumPy's rot90/fliplr) and (s, o) on the quantisation grid, makes
that candidate fit with zero residual (eq. 8).
"""
import numpy as np

from brute import transforms


def planted_image(H, W, n, step, bits, seed, plants):
    """plants: list of (range_index, (dy, dx), k, s, o).  Domains must not
    overlap any planted range.  Returns the image (uint16)."""
    rng = np.random.default_rng(seed)
    P = 1 << bits
    img = rng.integers(0, P, size=(H, W)).astype(np.int64)
    for (r, (dy, dx), k, s, o) in plants:
        Y, X = dy * step, dx * step
        # distinct cell values; multiples of 4 so that s * v stays integral
        vals = 4 * rng.permutation(np.arange(1, (P // 8)))[: n * n].reshape(n, n)
        img[Y:Y + 2 * n, X:X + 2 * n] = np.kron(vals, np.ones((2, 2), np.int64))
    for (r, (dy, dx), k, s, o) in plants:
        Y, X = dy * step, dx * step
        vals = img[Y:Y + 2 * n:2, X:X + 2 * n:2]
        b = s * transforms(vals)[k].astype(np.float64) + o
        assert np.all(b == np.floor(b)) and b.min() >= 0 and b.max() <= P - 1, "plant off range"
        ry, rx = divmod(r, W // n)
        assert not (ry * n < Y + 2 * n and Y < (ry + 1) * n and rx * n < X + 2 * n and X < (rx + 1) * n)
        img[ry * n:(ry + 1) * n, rx * n:(rx + 1) * n] = b.astype(np.int64)
    return img.astype(np.uint16)
