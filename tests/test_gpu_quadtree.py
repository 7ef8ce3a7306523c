"""Quadtree (adaptive range) encode on the GPU against the oracle's: the
same leaves, in the same order, with identical codes, element by element."""
import numpy as np
import pytest
import torch

import paper_1404_0774_amd as F
from oracle import oracle as O
from fic_inputs import gen_image

pytestmark = pytest.mark.gpu
LEAF = ("y", "x", "size", "domain", "iso", "s_idx", "o_idx", "err")


def gpu_quadtree(img, bits, n_max, n_min, step, tau, method=F.METHOD_MFMA, full=0):
    H, W = img.shape
    p = F.Params(H, W, bits, n_max, step, method=method, full_search=full)
    t = torch.from_numpy(np.ascontiguousarray(img).astype(np.uint8 if bits == 8 else np.int16)).cuda()
    out = F.encode_quadtree(t, p, n_min, tau)
    return {k: v.cpu().numpy() for k, v in out.items()}


def assert_leaves(got, ref, label):
    assert len(got["y"]) == len(ref["y"]), f"{label}: {len(got['y'])} leaves vs {len(ref['y'])}"
    for k in LEAF:
        if not np.array_equal(got[k], ref[k]):
            i = int(np.nonzero(got[k] != ref[k])[0][0])
            raise AssertionError(f"{label} {k}: first mismatch at leaf {i}: "
                                 + ", ".join(f"{q}={got[q][i]}/{ref[q][i]}" for q in LEAF))


@pytest.mark.parametrize("tau", [0.0, 20.0, 80.0, float("inf"), -1.0])
def test_decode_workload_quadtree_matches_oracle(tau):
    # 256x256 u8, ranges 8x8 split to 4x4 on the 4-pixel domain grid
    img = gen_image(256, 256, 8, 5)
    assert_leaves(gpu_quadtree(img, 8, 8, 4, 4, tau), O.encode_quadtree(img, 8, 4, 4, tau),
                  f"tau {tau}")


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("method", [F.METHOD_MFMA, F.METHOD_DIRECT])
@pytest.mark.parametrize("H,W,step,seed,tau", [(96, 80, 2, 61, 10.0), (64, 128, 4, 62, 30.0),
                                                (40, 56, 3, 63, 5.0)])
def test_small_quadtrees_match_oracle(method, full, H, W, step, seed, tau):
    if H % 8 or W % 8:
        pytest.skip("needs sides that are multiples of 8")
    img = gen_image(H, W, 8, seed)
    assert_leaves(gpu_quadtree(img, 8, 8, 4, step, tau, method, full),
                  O.encode_quadtree(img, 8, 4, step, tau), f"{H}x{W}")


def test_12bit_quadtree_matches_oracle():
    img = gen_image(128, 128, 12, 64)
    tau = 400.0
    assert_leaves(gpu_quadtree(img, 12, 8, 4, 2, tau),
                  O.encode_quadtree(img, 8, 4, 2, tau, bits=12), "12-bit")


def test_single_level_is_the_plain_encode():
    img = gen_image(128, 96, 8, 65)
    got = gpu_quadtree(img, 8, 8, 8, 4, 5.0)
    ref = O.encode(img, 8, 4)
    for k in ("domain", "iso", "s_idx", "o_idx", "err"):
        assert np.array_equal(got[k], ref[k]), k
    assert np.all(got["size"] == 8)


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("tau", [5.0, 40.0, -1.0])
def test_three_level_quadtree_matches_oracle(tau, full):
    # 16x16 ranges split into 8x8 and then 4x4
    img = gen_image(128, 128, 8, 66)
    assert_leaves(gpu_quadtree(img, 8, 16, 4, 4, tau, full=full),
                  O.encode_quadtree(img, 16, 4, 4, tau), f"16->4 tau {tau}")


def test_decode_workload_three_level_quadtree():
    img = gen_image(256, 256, 8, 5)
    assert_leaves(gpu_quadtree(img, 8, 16, 4, 4, 20.0), O.encode_quadtree(img, 16, 4, 4, 20.0),
                  "256 16->4")
