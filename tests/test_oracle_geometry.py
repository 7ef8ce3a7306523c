"""Pins for the oracle's block geometry: the contraction tau and the eight
transforms (Section V; Alg. 1), checked against NumPy's own routines and the
group structure of the square's symmetries."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O


def _generic(n, seed=0):
    # all entries distinct so every transform is distinguishable
    return np.random.default_rng(seed).permutation(n * n).reshape(n, n).astype(np.float64)


@pytest.mark.parametrize("n", [2, 3, 4, 8])
def test_isometries_match_numpy(n):
    b = _generic(n)
    f = np.fliplr(b)
    expect = [b, np.rot90(b, 1), np.rot90(b, 2), np.rot90(b, 3),
              f, np.rot90(f, 1), np.rot90(f, 2), np.rot90(f, 3)]
    for k in range(8):
        np.testing.assert_array_equal(O.isometry(b, k), expect[k])


@pytest.mark.parametrize("n", [4, 8])
def test_isometry_group_closure(n):
    b = _generic(n, 1)
    imgs = [O.isometry(b, k) for k in range(8)]
    # eight distinct blocks
    for p, q in itertools.combinations(range(8), 2):
        assert not np.array_equal(imgs[p], imgs[q])
    # closure: applying any transform to any transformed block gives one of the 8
    for p in range(8):
        for q in range(8):
            comp = O.isometry(imgs[p], q)
            assert sum(np.array_equal(comp, im) for im in imgs) == 1
    # identities of the dihedral group
    r = b
    for _ in range(4):
        r = O.isometry(r, 1)
    np.testing.assert_array_equal(r, b)                                  # rot90^4 = id
    np.testing.assert_array_equal(O.isometry(O.isometry(b, 4), 4), b)   # mirror^2 = id
    np.testing.assert_array_equal(O.isometry(O.isometry(O.isometry(b, 4), 1), 4),
                                  O.isometry(b, 3))                      # m r m = r^-1
    np.testing.assert_array_equal(O.isometry(b, 5), b.T)                 # transpose
    np.testing.assert_array_equal(O.isometry(b, 7), np.rot90(b, 2).T)    # anti-transpose
    # every element has an inverse within the set
    for p in range(8):
        assert any(np.array_equal(O.isometry(imgs[p], q), b) for q in range(8))


@pytest.mark.parametrize("n", [2, 4, 8])
def test_contract_is_2x2_mean(n):
    rng = np.random.default_rng(n)
    img = rng.integers(0, 4096, size=(40, 44)).astype(np.uint16)
    for (Y, X) in [(0, 0), (3, 5), (40 - 2 * n, 44 - 2 * n)]:
        ref = img[Y:Y + 2 * n, X:X + 2 * n].astype(np.float64).reshape(n, 2, n, 2).mean(axis=(1, 3))
        np.testing.assert_array_equal(O.contract(img, Y, X, n), ref)


def test_contract_commutes_with_transforms():
    # tau(S_k D) = S_k(tau D) for the 2n x 2n domain and the n x n result
    rng = np.random.default_rng(7)
    n = 4
    dom = rng.integers(0, 256, size=(2 * n, 2 * n)).astype(np.uint16)
    tD = O.contract(dom, 0, 0, n)
    for k in range(8):
        Sk_dom = O.isometry(dom.astype(np.float64), k).astype(np.uint16)
        np.testing.assert_array_equal(O.contract(Sk_dom, 0, 0, n), O.isometry(tD, k))


def test_grid_counts():
    # 512^2 with 8x8 ranges and 16x16 domains at stride 4: 4096 ranges, 125^2 domains
    assert O.n_ranges(512, 512, 8) == 4096
    assert O.n_domains(512, 512, 8, 4) == 15625
    # 256^2 with 4x4 ranges, 8x8 domains, stride 4: 64^2 ranges, 63^2 domains.
    # The related-work count of Section II (4096 ranges x 15,625 domains) is the
    # same range count; its domain count uses a different grid.
    assert O.n_ranges(256, 256, 4) == 4096
    assert O.n_domains(256, 256, 4, 4) == 63 * 63
    assert O.n_domains(512, 512, 8, 2) == 249 * 249
    assert O.n_domains(64, 64, 4, 4) == 225
