"""Pins for the oracle's decoder (iterating the PIFS map of eq. 6) and its
reverse-mode gradient: closed-form special cases, the contraction fixed point
(Section III-A), the collage bound (Section III-D) and finite differences."""
import numpy as np
import pytest

from oracle import oracle as O
from fic_inputs import gen_image
from brute import transforms


def random_codes(H, W, n, step, seed, smax=0.75):
    rng = np.random.default_rng(seed)
    R = (H // n) * (W // n)
    nd = O.n_domains(H, W, n, step)
    dom = rng.integers(0, nd, R).astype(np.int32)
    iso = rng.integers(0, 8, R).astype(np.uint8)
    s = rng.choice(np.arange(-smax, smax + 1e-9, 1 / 16), R)
    o = rng.integers(-64, 64, R) * 4.0
    return dom, iso, s, o


def map_matrix(H, W, n, step, dom, iso, s):
    """Dense matrix of x -> (s_r S_k tau x) built independently: the source
    cell of every range pixel comes from NumPy's rot90/fliplr of an index grid."""
    nx = (W - 2 * n) // step + 1
    M = np.zeros((H * W, H * W))
    idx = np.arange(n * n).reshape(n, n)
    for r in range(len(dom)):
        ry, rx = divmod(r, W // n)
        Y, X = (dom[r] // nx) * step, (dom[r] % nx) * step
        src = transforms(idx)[iso[r]]
        for i in range(n):
            for j in range(n):
                ci, cj = divmod(int(src[i, j]), n)
                p = (ry * n + i) * W + rx * n + j
                for (u, v) in ((0, 0), (0, 1), (1, 0), (1, 1)):
                    M[p, (Y + 2 * ci + u) * W + X + 2 * cj + v] += s[r] / 4.0
    return M


def range_const(H, W, n, vals):
    return np.kron(vals.reshape(H // n, W // n), np.ones((n, n)))


def test_zero_contrast_gives_offsets():
    H = W = 16; n = 4; step = 4
    dom, iso, s, o = random_codes(H, W, n, step, 0)
    s[:] = 0.0
    traj = O.decode(H, W, n, step, dom, iso, s, o, 5, 128.0)
    for t in range(1, 6):
        np.testing.assert_array_equal(traj[t], range_const(H, W, n, o))


def test_half_contrast_constant_offset_closed_form():
    H = W = 32; n = 4; step = 2
    dom, iso, s, o = random_codes(H, W, n, step, 1)
    s[:] = 0.5
    o[:] = 20.0
    traj = O.decode(H, W, n, step, dom, iso, s, o, 12, 128.0)
    for t in range(13):
        np.testing.assert_array_equal(traj[t], np.full((H, W), 40.0 + (128.0 - 40.0) / 2 ** t))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_converges_to_linear_fixed_point_within_contraction_bound(seed):
    H, W, n, step = 16, 24, 4, 2
    dom, iso, s, o = random_codes(H, W, n, step, 10 + seed)
    M = map_matrix(H, W, n, step, dom, iso, s)
    ovec = range_const(H, W, n, o).ravel()
    xstar = np.linalg.solve(np.eye(H * W) - M, ovec)
    T = 12
    traj = O.decode(H, W, n, step, dom, iso, s, o, T, 128.0)
    c = np.abs(s).max()
    for t in range(T + 1):
        # one application equals the independent matrix form
        if t < T:
            np.testing.assert_allclose(traj[t + 1].ravel(), M @ traj[t].ravel() + ovec, rtol=0, atol=1e-9)
        bound = c ** t * np.abs(128.0 - xstar).max()
        assert np.abs(traj[t].ravel() - xstar).max() <= bound * (1 + 1e-12) + 1e-9
    long = O.decode(H, W, n, step, dom, iso, s, o, 200, 128.0)
    np.testing.assert_allclose(long[-1].ravel(), xstar, rtol=0, atol=1e-8)


def test_collage_bound_on_encoded_image():
    # Collage theorem: the attractor is within ||f - W f|| / (1 - c) of f
    H = W = 32; n = 4; step = 4
    img = gen_image(H, W, 8, 3).astype(np.float64)
    codes = O.encode(img.astype(np.uint16), n, step)
    s, o = O.dequantize(codes["s_idx"], codes["o_idx"])
    s = np.clip(s, -0.875, 0.875)   # strictly contractive
    M = map_matrix(H, W, n, step, codes["domain"], codes["iso"], s)
    ovec = range_const(H, W, n, o).ravel()
    xstar = np.linalg.solve(np.eye(H * W) - M, ovec)
    Wf = O.pifs_apply(n, step, codes["domain"], codes["iso"], s, o, img)
    eps = np.abs(img - Wf).max()
    c = np.abs(s).max()
    assert np.abs(img.ravel() - xstar).max() <= eps / (1 - c) * (1 + 1e-9)


def _loss(H, W, n, step, dom, iso, s, o, T, target):
    x = O.decode(H, W, n, step, dom, iso, s, o, T, 128.0)[-1]
    return ((x - target) ** 2).mean()


def test_gradient_matches_central_differences():
    H = W = 16; n = 4; step = 2; T = 12
    dom, iso, s, o = random_codes(H, W, n, step, 5)
    target = gen_image(H, W, 8, 4).astype(np.float64)
    traj = O.decode(H, W, n, step, dom, iso, s, o, T, 128.0)
    g = 2.0 * (traj[-1] - target) / (H * W)
    gs, go = O.decode_backward(H, W, n, step, dom, iso, s, o, T, traj, g)
    hs, ho = 1e-5, 1e-3
    for r in range(len(s)):
        sp, sm = s.copy(), s.copy(); sp[r] += hs; sm[r] -= hs
        fd = (_loss(H, W, n, step, dom, iso, sp, o, T, target) - _loss(H, W, n, step, dom, iso, sm, o, T, target)) / (2 * hs)
        assert abs(fd - gs[r]) <= 1e-6 * max(1.0, abs(gs[r]))
        op, om = o.copy(), o.copy(); op[r] += ho; om[r] -= ho
        fd = (_loss(H, W, n, step, dom, iso, s, op, T, target) - _loss(H, W, n, step, dom, iso, s, om, T, target)) / (2 * ho)
        assert abs(fd - go[r]) <= 1e-8 * max(1.0, abs(go[r]))


def test_adjoint_dot_product_in_offsets():
    # x_T is affine in o for fixed s, so J_o v is an exact difference;
    # <J_o v, w> must equal <v, J_o^T w> from the reverse pass
    H, W, n, step, T = 16, 16, 4, 4, 12
    dom, iso, s, o = random_codes(H, W, n, step, 8)
    rng = np.random.default_rng(9)
    v = rng.standard_normal(len(o))
    w = rng.standard_normal((H, W))
    x1 = O.decode(H, W, n, step, dom, iso, s, o + v, T, 128.0)[-1]
    x0 = O.decode(H, W, n, step, dom, iso, s, o, T, 128.0)[-1]
    Jv = x1 - x0
    traj = O.decode(H, W, n, step, dom, iso, s, o, T, 128.0)
    gs, go = O.decode_backward(H, W, n, step, dom, iso, s, o, T, traj, w)
    lhs = (Jv * w).sum()
    rhs = (v * go).sum()
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
