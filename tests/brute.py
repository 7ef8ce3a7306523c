"""Brute-force encoder for tiny images, independent of the oracle.

It materialises every candidate block explicitly (NumPy slicing for the
domain, reshape-and-sum for the 2x2 contraction, ``np.rot90``/``np.fliplr``
for the eight transforms), fits by the centred (covariance) form of the least
squares line rather than the raw-moment form of eq. (9), and does everything
in exact integers: with S = 2^(s_bits-1) and the contracted value a = A/4,

    s*        = 4 sum (K A_i - SA)(K b_i - Sb) / sum (K A_i - SA)^2
    j         = floor((s* + 1) S + 1/2)            clamped to [0, 2S-1]
    o*        = mean(b) - s_q mean(a)
    m         = floor((o* + P)/delta_o + 1/2)      clamped to [0, 2^o_bits-1]
    16 S^2 E  = sum ((j - S) A_i + 4 S (o_q - b_i))^2

The winner is the lexicographic minimum of (E, c) over all candidates, taken
after the whole table is built (not as a running update).
"""
import numpy as np


def transforms(block):
    """The 8 blocks S_k(block), k = 0..7, from NumPy's own rot90/fliplr."""
    f = np.fliplr(block)
    return [block, np.rot90(block, 1), np.rot90(block, 2), np.rot90(block, 3),
            f, np.rot90(f, 1), np.rot90(f, 2), np.rot90(f, 3)]


def contract_sum(img, Y, X, n):
    """4 x tau: sums of the 2x2 cells of the 2n x 2n domain at (Y, X)."""
    blk = np.asarray(img[Y:Y + 2 * n, X:X + 2 * n], dtype=np.int64)
    return blk.reshape(n, 2, n, 2).sum(axis=(1, 3))


def _floor_div(a, b):
    return np.floor_divide(a, b)


def brute_encode(img, n, step, bits=8, s_bits=5, o_bits=7):
    img = np.asarray(img, dtype=np.int64)
    H, W = img.shape
    K = n * n
    P = 1 << bits
    S = 1 << (s_bits - 1)
    dlt = (2 * P) >> o_bits
    assert dlt * (1 << o_bits) == 2 * P
    ny, nx = (H - 2 * n) // step + 1, (W - 2 * n) // step + 1
    # candidate table (c = 8 d + k), each row K integer cell sums
    cands = []
    for dy in range(ny):
        for dx in range(nx):
            for t in transforms(contract_sum(img, dy * step, dx * step, n)):
                cands.append(np.ascontiguousarray(t).ravel())
    A = np.stack(cands).astype(np.int64)          # (C, K)
    SA = A.sum(1)
    cenA = K * A - SA[:, None]                    # K A_i - SA
    den = (cenA * cenA).sum(1)                    # K * D'
    R = (H // n) * (W // n)
    out = dict(domain=np.zeros(R, np.int32), iso=np.zeros(R, np.uint8),
               s_idx=np.zeros(R, np.uint8), o_idx=np.zeros(R, np.uint8),
               err=np.zeros(R, np.float64))
    for r in range(R):
        ry, rx = divmod(r, W // n)
        b = img[ry * n:(ry + 1) * n, rx * n:(rx + 1) * n].ravel().astype(np.int64)
        Sb = int(b.sum())
        cenb = K * b - Sb
        num = (cenA * cenb[None, :]).sum(1)       # K * N'
        # j = floor((4 num/den + 1) S + 1/2) = floor((8 S num + 2 S den + den) / (2 den))
        flat = den == 0
        dd = np.where(flat, 1, den)
        j = _floor_div(8 * S * num + 2 * S * dd + dd, 2 * dd)
        j = np.where(flat, S, j)                  # eq. (11): s = 0
        j = np.clip(j, 0, 2 * S - 1)
        js = j - S                                # s_q = js / S
        # o* = Sb/K - s_q SA/(4K);  (o* + P)/dlt + 1/2 = (4 S Sb - js SA + 4 S K P + 2 S K dlt) / (4 S K dlt)
        q = 4 * S * K * dlt
        m = _floor_div(4 * S * Sb - js * SA + 4 * S * K * P + 2 * S * K * dlt, q)
        m = np.clip(m, 0, (1 << o_bits) - 1)
        oq = m * dlt - P
        e = js[:, None] * A + 4 * S * (oq[:, None] - b[None, :])
        E16 = (e * e).sum(1)                      # 16 S^2 E, exact integer
        c = int(np.lexsort((np.arange(len(E16)), E16))[0])
        out["domain"][r] = c // 8
        out["iso"][r] = c % 8
        out["s_idx"][r] = j[c]
        out["o_idx"][r] = m[c]
        out["err"][r] = E16[c] / (16.0 * S * S)
    return out
