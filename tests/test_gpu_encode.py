"""GPU parity of the range-domain search (both kernels) against the CPU
oracle: identical codes and residuals, element by element."""
import numpy as np
import pytest
import torch

import paper_1404_0774_amd as F
from oracle import oracle as O
from fic_inputs import gen_image
from planted import planted_image, PLANTS_64_N8

pytestmark = pytest.mark.gpu
KEYS = ("domain", "iso", "s_idx", "o_idx", "err")
METHODS = [F.METHOD_MFMA, F.METHOD_DIRECT]


def gpu_encode(img, n, step, bits, method, ranges=None, full=0):
    H, W = img.shape
    p = F.Params(H, W, bits, n, step, method=method, full_search=full)
    dt = torch.uint8 if bits == 8 else torch.int16
    t = torch.from_numpy(np.ascontiguousarray(img).astype(np.uint8 if bits == 8 else np.int16)).to("cuda")
    out = F.encode(t, p)
    torch.cuda.synchronize()
    res = {k: out[k].cpu().numpy() for k in KEYS}
    if ranges is not None:
        res = {k: v[ranges] for k, v in res.items()}
    return res


def assert_same(gpu, ora, label=""):
    for k in KEYS:
        if not np.array_equal(gpu[k], ora[k]):
            bad = np.nonzero(gpu[k] != ora[k])[0]
            i = bad[0]
            raise AssertionError(f"{label} {k}: {len(bad)} mismatches, first at {i}: "
                                 + ", ".join(f"{q}={gpu[q][i]}/{ora[q][i]}" for q in KEYS))


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("method", METHODS)
def test_plain_64x64_config(method, full):
    # 64x64 u8, 4x4 ranges, 8x8 domains at stride 4: the plain full-search setup
    img = gen_image(64, 64, 8, 1)
    assert_same(gpu_encode(img, 4, 4, 8, method, full=full), O.encode(img, 4, 4), "plain64")


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("H,W,n,step,seed", [
    (96, 80, 4, 2, 11),     # 480 ranges (ragged tile), 1665 domains (ragged block)
    (128, 96, 8, 4, 12),    # n = 8, 192 ranges, 609 domains
    (40, 56, 4, 3, 13),     # odd stride
    (8, 8, 4, 4, 14),       # smallest image: 4 ranges, one domain
    (16, 64, 8, 1, 15),     # one domain row, stride 1
])
def test_parity_small_images(method, H, W, n, step, seed, full):
    img = gen_image(H, W, 8, seed)
    assert_same(gpu_encode(img, n, step, 8, method, full=full), O.encode(img, n, step),
                f"{H}x{W}")


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("method", METHODS + [F.METHOD_MFMA_I8])
@pytest.mark.parametrize("bits", [8, 12])
def test_search_visits_exactly_the_ranges_and_domains_with_variance(bits, method, full):
    """Without full_search both searches skip flat ranges and flat domains
    (their outcome is fixed); with it they visit every range and domain.  The
    counts they report match a direct count."""
    if method == F.METHOD_MFMA_I8 and bits == 8:
        pytest.skip("the int8 search takes 12-bit images")
    H, W, n, step = 128, 96, 8, 4
    img = gen_image(H, W, bits, 19)
    p = F.Params(H, W, bits, n, step, method=method, full_search=full)
    host = img.astype(np.uint8 if bits == 8 else np.int16)
    out = F.encode(torch.from_numpy(host).cuda(), p)
    nr, nd = F.search_counts(out, p)
    blocks = img.reshape(H // n, n, W // n, n).transpose(0, 2, 1, 3).reshape(-1, n * n)
    want_r = int((blocks.max(1) != blocks.min(1)).sum())
    ny, nx = (H - 2 * n) // step + 1, (W - 2 * n) // step + 1
    cells = [img[y * step:y * step + 2 * n, x * step:x * step + 2 * n]
             .reshape(n, 2, n, 2).astype(np.int64).sum(axis=(1, 3))
             for y in range(ny) for x in range(nx)]
    want_d = sum(int(c.max() != c.min()) for c in cells)
    assert 0 < want_r < len(blocks) and 0 < want_d < ny * nx   # the image has background
    if full:
        assert (nr, nd) == (len(blocks), ny * nx)
    else:
        assert (nr, nd) == (want_r, want_d)
    assert_same({k: out[k].cpu().numpy() for k in KEYS}, O.encode(img, n, step, bits=bits),
                f"counts image {bits}-bit")


def test_unaligned_image_takes_range_operand_path():
    """8x8 ranges normally build the range fragments from the image; an image
    that is not 8-byte aligned goes through the range operand instead.  Both
    give the oracle's codes."""
    H, W, n, step = 96, 128, 8, 4
    img = gen_image(H, W, 8, 17)
    p = F.Params(H, W, 8, n, step)
    buf = torch.zeros(H * W + 8, dtype=torch.uint8, device="cuda")
    res = []
    for off in (0, 3):
        view = buf[off:off + H * W].view(H, W)
        view.copy_(torch.from_numpy(img))
        assert (view.data_ptr() % 8 == 0) == (off == 0)
        out = F.encode(view, p)
        torch.cuda.synchronize()
        res.append({k: out[k].cpu().numpy() for k in KEYS})
    ora = O.encode(img, n, step)
    assert_same(res[0], ora, "aligned")
    assert_same(res[1], ora, "unaligned")


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("kind", ["zeros", "const", "max", "checker", "noise", "levels"])
def test_parity_degenerate_images(method, kind, full):
    H = W = 48
    rng = np.random.default_rng(5)
    img = {"zeros": np.zeros((H, W)), "const": np.full((H, W), 101),
           "max": np.full((H, W), 255),
           "checker": (np.indices((H, W)).sum(0) % 2) * 255,
           "noise": rng.integers(0, 256, (H, W)),
           "levels": rng.integers(0, 3, (H, W)) * 85}[kind].astype(np.uint8)
    for (n, step) in [(4, 4), (8, 2)]:
        assert_same(gpu_encode(img, n, step, 8, method, full=full), O.encode(img, n, step), kind)


@pytest.mark.parametrize("method", METHODS)
def test_planted_codes(method):
    H = W = 64
    n, step = 8, 4
    plants = PLANTS_64_N8
    img = planted_image(H, W, n, step, 8, 23, plants).astype(np.uint8)
    gpu = gpu_encode(img, n, step, 8, method)
    assert_same(gpu, O.encode(img, n, step), "planted")
    nx = (W - 2 * n) // step + 1
    for (r, (dy, dx), k, s, o) in plants:
        assert gpu["err"][r] == 0.0 and gpu["domain"][r] == dy * nx + dx and gpu["iso"][r] == k


# Oracle tables of the full-size workloads, computed once per session (the
# oracle is plain C over all host threads: ~5 s for 512x512 u8 at stride 4,
# ~20 s for 512x512 12-bit at stride 2 on 16 threads).
_ORACLE = {}


def oracle_table(key, img, n, step, bits=8):
    if key not in _ORACLE:
        _ORACLE[key] = O.encode(img, n, step, bits=bits)
    return _ORACLE[key]


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("method", METHODS)
def test_u8_512_every_range_matches_oracle(method, full):
    # 512x512 u8, 8x8 ranges, 16x16 domains at stride 4 (4096 x 125,000
    # candidates): all 4096 codes element by element
    img = gen_image(512, 512, 8, 2)
    got = gpu_encode(img, 8, 4, 8, method, full=full)
    assert_same(got, oracle_table("u8_512", img, 8, 4), f"u8_512 method {method} full {full}")


@pytest.mark.parametrize("full", [0, 1])
def test_decode_workload_encode_matches_oracle(full):
    # 256x256 u8, 4x4 ranges, 8x8 domains at stride 4
    img = gen_image(256, 256, 8, 5)
    got = gpu_encode(img, 4, 4, 8, F.METHOD_MFMA, full=full)
    assert_same(got, oracle_table("u8_256_n4", img, 4, 4), "decode256")


def test_deterministic_repeat():
    img = gen_image(128, 128, 8, 9)
    a = gpu_encode(img, 8, 2, 8, F.METHOD_MFMA)
    for _ in range(3):
        assert_same(gpu_encode(img, 8, 2, 8, F.METHOD_MFMA), a, "repeat")


# --- 12-bit images: hi/lo split contraction ---------------------------------

METHODS12 = METHODS + [F.METHOD_MFMA_I8]


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("method", METHODS12)
@pytest.mark.parametrize("H,W,n,step,seed", [
    (48, 64, 4, 2, 41),     # 192 ranges, ragged tiles
    (64, 64, 8, 4, 42),
    (40, 56, 4, 3, 43),
    (96, 80, 8, 2, 44),     # 120 ranges (ragged tile), 1,161 domains
])
def test_parity_12bit_small(method, H, W, n, step, seed, full):
    if method == F.METHOD_MFMA_I8 and n != 8:
        pytest.skip("the int8 search takes 8x8 ranges")
    img = gen_image(H, W, 12, seed)
    assert_same(gpu_encode(img, n, step, 12, method, full=full), O.encode(img, n, step, bits=12),
                f"12b {H}x{W}")


@pytest.fixture
def restore_tuning():
    yield
    F.set_tuning([])
    F.load_tuning(F._lib.TUNING_PATH)


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("method", [F.METHOD_MFMA, F.METHOD_MFMA_I8])
def test_12bit_launch_shapes_give_oracle_codes(method, full, restore_tuning):
    """Every chunk count gives the oracle's codes: one chunk per row group,
    chunks that do not divide the column blocks, the tuned 24, and more than
    there are blocks (clamped); without the full flag fewer row groups are
    searched than the grid holds, and the workgroups left over return."""
    img = gen_image(96, 80, 12, 44)   # 120 ranges, 1,353 domains (43 blocks)
    ref = O.encode(img, 8, 2, bits=12)
    for chunks in (1, 5, 24, 200):
        F.set_tuning([dict(bit_depth=12, range_size=8, method=method, min_domains=0,
                           col_chunks=chunks, seed_blocks=1)])
        assert_same(gpu_encode(img, 8, 2, 12, method, full=full), ref,
                    f"12b chunks={chunks}")


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("method", METHODS12)
@pytest.mark.parametrize("kind", ["zeros", "max", "noise", "checker"])
def test_parity_12bit_degenerate(method, kind, full):
    H = W = 48
    rng = np.random.default_rng(7)
    img = {"zeros": np.zeros((H, W)), "max": np.full((H, W), 4095),
           "noise": rng.integers(0, 4096, (H, W)),
           "checker": (np.indices((H, W)).sum(0) % 2) * 4095}[kind].astype(np.uint16)
    for (n, step) in [(4, 4), (8, 2)]:
        if method == F.METHOD_MFMA_I8 and n != 8:
            continue
        assert_same(gpu_encode(img, n, step, 12, method, full=full),
                    O.encode(img, n, step, bits=12), kind)


@pytest.mark.parametrize("method", METHODS)
def test_planted_codes_12bit(method):
    H = W = 32
    n, step, P = 4, 4, 4096
    plants = [(63, (0, 0), 1, 0.5, 8.0 * 16), (56, (0, 5), 4, -0.5, P / 2.0),
              (7, (5, 0), 6, 0.75, 0.0), (35, (1, 1), 3, 0.25, P / 4.0)]
    img = planted_image(H, W, n, step, 12, 29, plants)
    gpu = gpu_encode(img, n, step, 12, method)
    assert_same(gpu, O.encode(img, n, step, bits=12), "planted12")
    nx = (W - 2 * n) // step + 1
    for (r, (dy, dx), k, s, o) in plants:
        assert gpu["err"][r] == 0.0 and gpu["domain"][r] == dy * nx + dx and gpu["iso"][r] == k


@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("method", METHODS12)
def test_ct12_512_every_range_matches_oracle(method, full):
    # 512x512 12-bit, 8x8 ranges, 16x16 domains at stride 2 (4096 x 496,008
    # candidates): all 4096 codes element by element
    img = gen_image(512, 512, 12, 3)
    got = gpu_encode(img, 8, 2, 12, method, full=full)
    assert_same(got, oracle_table("ct12_512", img, 8, 2, bits=12),
                f"ct12_512 method {method} full {full}")


@pytest.mark.parametrize("method", [F.METHOD_MFMA, F.METHOD_MFMA_I8])
def test_planted_codes_12bit_n8(method):
    """Planted exact 8x8 ranges in a 12-bit image: residual 0 and the planted
    code, on both matrix-core searches."""
    H = W = 64
    n, step = 8, 4
    P = 4096
    plants = [(56, (0, 0), 5, 0.5, 64.0 * 8), (63, (1, 2), 2, -0.25, P / 2.0)]
    img = planted_image(H, W, n, step, 12, 31, plants)
    gpu = gpu_encode(img, n, step, 12, method)
    assert_same(gpu, O.encode(img, n, step, bits=12), "planted12 n8")
    nx = (W - 2 * n) // step + 1
    for (r, (dy, dx), k, s, o) in plants:
        assert gpu["err"][r] == 0.0 and gpu["domain"][r] == dy * nx + dx and gpu["iso"][r] == k


def test_int8_search_refuses_8bit_and_4x4():
    for p in (F.Params(64, 64, 8, 8, 4, method=F.METHOD_MFMA_I8),
              F.Params(64, 64, 12, 4, 4, method=F.METHOD_MFMA_I8)):
        img = torch.zeros((64, 64), dtype=torch.uint8 if p.bit_depth == 8 else torch.uint16,
                          device="cuda")
        with pytest.raises(F.FicError) as e:
            F.encode(img, p)
        assert e.value.status == 2


# --- 16x16 ranges (8-bit, centred FP16 operands) ------------------------------

@pytest.mark.parametrize("full", [0, 1])
@pytest.mark.parametrize("H,W,step,seed", [(64, 64, 8, 71), (128, 96, 4, 72), (96, 160, 2, 73)])
def test_16x16_ranges_match_oracle(H, W, step, seed, full):
    img = gen_image(H, W, 8, seed)
    assert_same(gpu_encode(img, 16, step, 8, F.METHOD_MFMA, full=full), O.encode(img, 16, step),
                f"n16 {H}x{W}")


@pytest.mark.parametrize("kind", ["zeros", "max", "checker", "noise", "halves"])
def test_16x16_ranges_degenerate_and_extreme_images(kind):
    # "max" and "checker" put the centred sums at their bounds
    H = W = 64
    rng = np.random.default_rng(8)
    img = {"zeros": np.zeros((H, W)), "max": np.full((H, W), 255),
           "checker": (np.indices((H, W)).sum(0) % 2) * 255,
           "noise": rng.integers(0, 256, (H, W)),
           "halves": np.where(np.arange(W)[None, :] < W // 2, 255, 0) * np.ones((H, 1))
           }[kind].astype(np.uint8)
    for full in (0, 1):
        assert_same(gpu_encode(img, 16, 8, 8, F.METHOD_MFMA, full=full), O.encode(img, 16, 8), kind)


def test_16x16_ranges_refuse_the_plain_method_and_12bit():
    for bits, method in ((8, F.METHOD_DIRECT), (12, F.METHOD_MFMA)):
        p = F.Params(64, 64, bits, 16, 8, method=method)
        img = torch.zeros((64, 64), dtype=torch.uint8 if bits == 8 else torch.uint16, device="cuda")
        with pytest.raises(F.FicError) as e:
            F.encode(img, p)
        assert e.value.status == 2
