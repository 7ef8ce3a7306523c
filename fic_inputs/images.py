"""Synthetic CT/MR-like test images (seeded, deterministic).

Recipe (all draws from ``numpy.random.default_rng(seed)`` in this order):

1. Texture: white noise N(0, 1) of shape (H, W), blurred by a separable
   Gaussian (sigma 4, radius 16, reflect boundary), min-max scaled to [0, 1]
   and quantised to 40 levels: ``tex = clip(floor(40 t), 0, 39)``.
2. Body: an ellipse centred at (H/2, W/2) jittered by up to +-5 % of each side,
   with semi-axes U[0.38, 0.46] * (H, W).  Outside it the image is exactly 0.
3. Lesions: ``integers(3, 9)`` filled, rotated ellipses (later ones overwrite
   earlier ones), centres inside the body by rejection sampling, semi-axes
   U[0.04, 0.18] * min(H, W), angle U[0, pi).  Fill value v:
   8-bit ``integers(60, 221)``; 12-bit ``integers(0, 4096)``.
4. 8-bit pixel inside the body: ``clip(v_or_0 + tex, 0, 255)`` stored as uint8.
5. 12-bit pixel inside the body: ``round(v_or_0 + 16 tex + N(0, 20^2))``
   clipped to [0, 4095], stored as uint16 (noise drawn for every pixel, applied
   inside the body only).

Per-workload seeds: plain 64x64 search 1, 512x512 8-bit 2, 512x512 12-bit 3,
256x256 decode workload 5; the 64-slice batch draws its sides from
``default_rng(4)`` and slice i uses seed 4000 + i.
"""
import numpy as np

BATCH_SIDES = (256, 320, 384, 448, 512)
CONFIG_SEEDS = {"plain64": 1, "u8_512": 2, "ct12_512": 3, "batch": 4, "decode256": 5}


def _gauss_kernel(sigma: float, radius: int) -> np.ndarray:
    x = np.arange(-radius, radius + 1, dtype=np.float64)
    k = np.exp(-0.5 * (x / sigma) ** 2)
    return k / k.sum()


def _blur_axis(a: np.ndarray, k: np.ndarray, axis: int) -> np.ndarray:
    r = (len(k) - 1) // 2
    pad = [(0, 0), (0, 0)]
    pad[axis] = (r, r)
    p = np.pad(a, pad, mode="reflect") if a.shape[axis] > r else np.pad(a, pad, mode="symmetric")
    out = np.zeros_like(a)
    n = a.shape[axis]
    for i, w in enumerate(k):
        sl = [slice(None), slice(None)]
        sl[axis] = slice(i, i + n)
        out += w * p[tuple(sl)]
    return out


def gen_image(height: int, width: int, bits: int = 8, seed: int = 0) -> np.ndarray:
    """Return one synthetic slice, uint8 (bits=8) or uint16 (bits=12), shape (H, W)."""
    if bits not in (8, 12):
        raise ValueError("bits must be 8 or 12")
    if height < 1 or width < 1:
        raise ValueError("empty image")
    rng = np.random.default_rng(seed)
    H, W = int(height), int(width)

    # 1. texture
    w = rng.standard_normal((H, W))
    k = _gauss_kernel(4.0, 16)
    t = _blur_axis(_blur_axis(w, k, 0), k, 1)
    lo, hi = t.min(), t.max()
    t = (t - lo) / (hi - lo) if hi > lo else np.zeros_like(t)
    tex = np.clip(np.floor(40.0 * t), 0, 39)

    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    # 2. body mask
    cy = H / 2.0 + rng.uniform(-0.05, 0.05) * H
    cx = W / 2.0 + rng.uniform(-0.05, 0.05) * W
    ay = rng.uniform(0.38, 0.46) * H
    ax = rng.uniform(0.38, 0.46) * W
    body = ((yy - cy) / ay) ** 2 + ((xx - cx) / ax) ** 2 <= 1.0

    # 3. lesions
    fill = np.zeros((H, W), dtype=np.float64)
    n_les = int(rng.integers(3, 9))
    m = float(min(H, W))
    for _ in range(n_les):
        for _attempt in range(1000):
            ly = rng.uniform(0, H)
            lx = rng.uniform(0, W)
            if ((ly - cy) / ay) ** 2 + ((lx - cx) / ax) ** 2 <= 1.0:
                break
        sy = rng.uniform(0.04, 0.18) * m
        sx = rng.uniform(0.04, 0.18) * m
        ang = rng.uniform(0.0, np.pi)
        v = int(rng.integers(60, 221)) if bits == 8 else int(rng.integers(0, 4096))
        c, s = np.cos(ang), np.sin(ang)
        u = (xx - lx) * c + (yy - ly) * s
        q = -(xx - lx) * s + (yy - ly) * c
        fill[(u / sx) ** 2 + (q / sy) ** 2 <= 1.0] = v

    if bits == 8:
        img = np.clip(fill + tex, 0, 255)
        img[~body] = 0
        return img.astype(np.uint8)
    noise = rng.normal(0.0, 20.0, size=(H, W))
    img = np.clip(np.rint(fill + 16.0 * tex + noise), 0, 4095)
    img[~body] = 0
    return img.astype(np.uint16)


def batch_sides(n_slices: int = 64, seed: int = CONFIG_SEEDS["batch"]) -> list:
    """Side lengths of the uneven batch: uniform over BATCH_SIDES."""
    rng = np.random.default_rng(seed)
    return [int(BATCH_SIDES[i]) for i in rng.integers(0, len(BATCH_SIDES), size=n_slices)]
