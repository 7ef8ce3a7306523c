"""ctypes wrapper around liboracle.so (test infrastructure only).

Every function takes and returns NumPy arrays.  Images are passed as uint16
(uint8 inputs are widened, which is marshalling only).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        i32, i64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        p = ctypes.c_void_p
        L.oracle_n_ranges.restype = i64
        L.oracle_n_ranges.argtypes = [i32, i32, i32]
        L.oracle_n_domains.restype = i64
        L.oracle_n_domains.argtypes = [i32, i32, i32, i32]
        L.oracle_contract.restype = None
        L.oracle_contract.argtypes = [p, i32, i32, i32, i32, p]
        L.oracle_isometry.restype = None
        L.oracle_isometry.argtypes = [p, i32, i32, p]
        L.oracle_fit.restype = None
        L.oracle_fit.argtypes = [p, p, i32, i32, i32, i32, p, p, p, p, p]
        L.oracle_encode.restype = i32
        L.oracle_encode.argtypes = [i32, i32, i32, i32, i32, i32, i32, p, i64, i64, i32,
                                    p, p, p, p, p]
        L.oracle_encode_list.restype = i32
        L.oracle_encode_list.argtypes = [i32, i32, i32, i32, i32, i32, i32, p, p, i64, i32,
                                         p, p, p, p, p]
        L.oracle_decode.restype = i32
        L.oracle_decode.argtypes = [i32, i32, i32, i32, p, p, p, p, i32, dbl, p]
        L.oracle_decode_scaled.restype = i32
        L.oracle_decode_scaled.argtypes = [i32, i32, i32, i32, i32, i32, p, p, p, p, i32, dbl, p]
        L.oracle_decode_backward.restype = i32
        L.oracle_decode_backward.argtypes = [i32, i32, i32, i32, p, p, p, p, i32, p, p, p, p]
        L.oracle_pifs_apply.restype = i32
        L.oracle_pifs_apply.argtypes = [i32, i32, i32, i32, p, p, p, p, p, p]
        L.oracle_stream_domain_bits.restype = i32
        L.oracle_stream_domain_bits.argtypes = [i64]
        L.oracle_stream_bytes.restype = i64
        L.oracle_stream_bytes.argtypes = [i32, i32, i32, i32, i32, i32]
        L.oracle_stream_pack.restype = i32
        L.oracle_stream_pack.argtypes = [i32, i32, i32, i32, i32, i32, i32, p, p, p, p, p, i64]
        L.oracle_stream_unpack.restype = i32
        L.oracle_stream_unpack.argtypes = [i32, i32, i32, i32, i32, i32, p, i64, p, p, p, p]
        L.oracle_max_threads.restype = i32
        L.oracle_max_threads.argtypes = []
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def n_ranges(h, w, n):
    return int(lib().oracle_n_ranges(h, w, n))


def n_domains(h, w, n, step):
    return int(lib().oracle_n_domains(h, w, n, step))


def domain_grid(h, w, n, step):
    """(ny, nx): number of domain positions along each axis."""
    ny = (h - 2 * n) // step + 1 if h >= 2 * n else 0
    nx = (w - 2 * n) // step + 1 if w >= 2 * n else 0
    return ny, nx


def contract(img, Y, X, n):
    img = np.ascontiguousarray(img, dtype=np.uint16)
    out = np.zeros((n, n), np.float64)
    lib().oracle_contract(_ptr(img), img.shape[1], Y, X, n, _ptr(out))
    return out


def isometry(block, k):
    block = np.ascontiguousarray(block, dtype=np.float64)
    n = block.shape[0]
    out = np.zeros_like(block)
    lib().oracle_isometry(_ptr(block), n, k, _ptr(out))
    return out


def fit(a, b, bits=8, s_bits=5, o_bits=7):
    """Fit one K-pixel pair; returns (j, m, s_q, o_q, err)."""
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    j = np.zeros(1, np.int32); m = np.zeros(1, np.int32)
    s = np.zeros(1); o = np.zeros(1); e = np.zeros(1)
    lib().oracle_fit(_ptr(a), _ptr(b), a.size, bits, s_bits, o_bits,
                     _ptr(j), _ptr(m), _ptr(s), _ptr(o), _ptr(e))
    return int(j[0]), int(m[0]), float(s[0]), float(o[0]), float(e[0])


def encode(img, n, step, bits=8, s_bits=5, o_bits=7, r_begin=0, r_end=None, threads=0):
    """Full search over ranges [r_begin, r_end); returns dict of SoA arrays."""
    img = np.ascontiguousarray(img, dtype=np.uint16)
    H, W = img.shape
    R = n_ranges(H, W, n)
    if r_end is None:
        r_end = R
    cnt = r_end - r_begin
    out = dict(domain=np.zeros(cnt, np.int32), iso=np.zeros(cnt, np.uint8),
               s_idx=np.zeros(cnt, np.uint8), o_idx=np.zeros(cnt, np.uint8),
               err=np.zeros(cnt, np.float64))
    rc = lib().oracle_encode(H, W, bits, n, step, s_bits, o_bits, _ptr(img), r_begin, r_end,
                             threads, _ptr(out["domain"]), _ptr(out["iso"]), _ptr(out["s_idx"]),
                             _ptr(out["o_idx"]), _ptr(out["err"]))
    if rc != 0:
        raise ValueError("oracle_encode: invalid parameters")
    return out


def encode_ranges(img, n, step, ranges, bits=8, s_bits=5, o_bits=7, threads=0):
    """Full search for the listed range indices; returns dict of SoA arrays."""
    img = np.ascontiguousarray(img, dtype=np.uint16)
    H, W = img.shape
    rs = np.ascontiguousarray(ranges, dtype=np.int64)
    cnt = len(rs)
    out = dict(domain=np.zeros(cnt, np.int32), iso=np.zeros(cnt, np.uint8),
               s_idx=np.zeros(cnt, np.uint8), o_idx=np.zeros(cnt, np.uint8),
               err=np.zeros(cnt, np.float64))
    rc = lib().oracle_encode_list(H, W, bits, n, step, s_bits, o_bits, _ptr(img), _ptr(rs), cnt,
                                  threads, _ptr(out["domain"]), _ptr(out["iso"]),
                                  _ptr(out["s_idx"]), _ptr(out["o_idx"]), _ptr(out["err"]))
    if rc != 0:
        raise ValueError("oracle_encode_list: invalid parameters")
    return out


def quadtree_sizes(n_max, n_min):
    """Range sides of the levels: n_max, n_max / 2, ..., n_min."""
    sizes = [n_max]
    while sizes[-1] > n_min:
        sizes.append(sizes[-1] // 2)
    if sizes[-1] != n_min:
        raise ValueError("n_min must be n_max divided by a power of two")
    return sizes


def encode_quadtree(img, n_max, n_min, step, tau, bits=8, s_bits=5, o_bits=7):
    """Adaptive partition of the range blocks (Section V's quadtree method;
    Section II's adaptive fractal coding).  Reading used here: every range
    of side n_max is encoded by the full search (domains of side 2 n on the
    STEP grid, the same for every level); a range whose residual (eq. 8 with
    the quantised s, o) exceeds tau * n^2, tau a squared error per pixel,
    and whose side is above n_min is split into its four quadrants, which
    are encoded the same way at side n / 2.  The leaves are listed top-level
    range by top-level range (row-major), each one's leaves in Z order
    (top-left, top-right, bottom-left, bottom-right, recursively).

    Returns a dict of leaf arrays (y, x, size, domain, iso, s_idx, o_idx,
    err) and `split`, per level above n_min, the split flag of every range
    of that level's grid (0 for ranges that were not encoded)."""
    img = np.ascontiguousarray(img, dtype=np.uint16)
    H, W = img.shape
    sizes = quadtree_sizes(n_max, n_min)
    if H % n_max or W % n_max:
        raise ValueError("image sides must be multiples of n_max")
    codes = {}      # (y, x, n) -> (domain, iso, s_idx, o_idx, err)
    split = []
    active = [(ry * n_max, rx * n_max) for ry in range(H // n_max) for rx in range(W // n_max)]
    for n in sizes:
        rw = W // n
        idx = np.array([(y // n) * rw + x // n for (y, x) in active], np.int64)
        c = encode_ranges(img, n, step, idx, bits, s_bits, o_bits)
        for i, (y, x) in enumerate(active):
            codes[(y, x, n)] = (int(c["domain"][i]), int(c["iso"][i]), int(c["s_idx"][i]),
                                int(c["o_idx"][i]), float(c["err"][i]))
        if n == n_min:
            break
        flags = np.zeros((H // n) * rw, np.uint8)
        nxt = []
        for i, (y, x) in enumerate(active):
            if c["err"][i] > tau * (n * n):
                flags[(y // n) * rw + x // n] = 1
                h = n // 2
                nxt += [(y, x), (y, x + h), (y + h, x), (y + h, x + h)]
        split.append(flags)
        active = nxt
    leaves = []

    def walk(y, x, n, level):
        if level < len(split) and split[level][(y // n) * (W // n) + x // n]:
            h = n // 2
            for (dy, dx) in ((0, 0), (0, h), (h, 0), (h, h)):
                walk(y + dy, x + dx, h, level + 1)
        else:
            leaves.append((y, x, n) + codes[(y, x, n)])

    for ry in range(H // n_max):
        for rx in range(W // n_max):
            walk(ry * n_max, rx * n_max, n_max, 0)
    cols = list(zip(*leaves))
    out = dict(y=np.array(cols[0], np.int32), x=np.array(cols[1], np.int32),
               size=np.array(cols[2], np.uint8), domain=np.array(cols[3], np.int32),
               iso=np.array(cols[4], np.uint8), s_idx=np.array(cols[5], np.uint8),
               o_idx=np.array(cols[6], np.uint8), err=np.array(cols[7], np.float64))
    out["split"] = split
    return out


def dequantize(s_idx, o_idx, bits=8, s_bits=5, o_bits=7):
    """Grid values of the quantised codes (same grid definition as the oracle's fit)."""
    s = np.asarray(s_idx, np.float64) / 2.0 ** (s_bits - 1) - 1.0
    P = 2.0 ** bits
    o = np.asarray(o_idx, np.float64) * (2.0 * P / 2.0 ** o_bits) - P
    return s, o


def pifs_apply(n, step, domain, iso, s, o, x):
    x = np.ascontiguousarray(x, np.float64)
    h, w = x.shape
    y = np.zeros_like(x)
    rc = lib().oracle_pifs_apply(h, w, n, step, _ptr(np.ascontiguousarray(domain, np.int32)),
                                 _ptr(np.ascontiguousarray(iso, np.uint8)),
                                 _ptr(np.ascontiguousarray(s, np.float64)),
                                 _ptr(np.ascontiguousarray(o, np.float64)), _ptr(x), _ptr(y))
    if rc != 0:
        raise ValueError("oracle_pifs_apply: invalid parameters")
    return y


def decode(h, w, n, step, domain, iso, s, o, iters, x0):
    domain = np.ascontiguousarray(domain, np.int32)
    iso = np.ascontiguousarray(iso, np.uint8)
    s = np.ascontiguousarray(s, np.float64)
    o = np.ascontiguousarray(o, np.float64)
    traj = np.zeros((iters + 1, h, w), np.float64)
    rc = lib().oracle_decode(h, w, n, step, _ptr(domain), _ptr(iso), _ptr(s), _ptr(o),
                             iters, float(x0), _ptr(traj))
    if rc != 0:
        raise ValueError("oracle_decode: invalid parameters")
    return traj


def decode_scaled(h, w, n, step, num, den, domain, iso, s, o, iters, x0):
    """Decode the codes of an h x w image at scale num/den; returns the
    trajectory (iters+1, h*num/den, w*num/den)."""
    domain = np.ascontiguousarray(domain, np.int32)
    iso = np.ascontiguousarray(iso, np.uint8)
    s = np.ascontiguousarray(s, np.float64)
    o = np.ascontiguousarray(o, np.float64)
    if (h * num) % den or (w * num) % den:
        raise ValueError("decode_scaled: the scaled image is not whole pixels")
    traj = np.zeros((iters + 1, h * num // den, w * num // den), np.float64)
    rc = lib().oracle_decode_scaled(h, w, n, step, num, den, _ptr(domain), _ptr(iso), _ptr(s),
                                    _ptr(o), iters, float(x0), _ptr(traj))
    if rc != 0:
        raise ValueError("oracle_decode_scaled: invalid parameters")
    return traj


def decode_backward(h, w, n, step, domain, iso, s, o, iters, traj, grad_xT):
    domain = np.ascontiguousarray(domain, np.int32)
    iso = np.ascontiguousarray(iso, np.uint8)
    s = np.ascontiguousarray(s, np.float64)
    o = np.ascontiguousarray(o, np.float64)
    traj = np.ascontiguousarray(traj, np.float64)
    g = np.ascontiguousarray(grad_xT, np.float64)
    R = n_ranges(h, w, n)
    gs = np.zeros(R); go = np.zeros(R)
    rc = lib().oracle_decode_backward(h, w, n, step, _ptr(domain), _ptr(iso), _ptr(s), _ptr(o),
                                      iters, _ptr(traj), _ptr(g), _ptr(gs), _ptr(go))
    if rc != 0:
        raise ValueError("oracle_decode_backward: invalid parameters")
    return gs, go


def stream_domain_bits(n_domains):
    return int(lib().oracle_stream_domain_bits(int(n_domains)))


def stream_bytes(h, w, n, step, s_bits=5, o_bits=7):
    return int(lib().oracle_stream_bytes(h, w, n, step, s_bits, o_bits))


def stream_pack(h, w, n, step, codes, bits=8, s_bits=5, o_bits=7):
    """The code stream (header and records) of a dict of code arrays, as bytes."""
    nb = stream_bytes(h, w, n, step, s_bits, o_bits)
    out = np.zeros(nb, np.uint8)
    arr = [np.ascontiguousarray(codes["domain"], np.int32), np.ascontiguousarray(codes["iso"], np.uint8),
           np.ascontiguousarray(codes["s_idx"], np.uint8), np.ascontiguousarray(codes["o_idx"], np.uint8)]
    rc = lib().oracle_stream_pack(h, w, bits, n, step, s_bits, o_bits, *[_ptr(a) for a in arr],
                                  _ptr(out), nb)
    if rc != 0:
        raise ValueError("oracle_stream_pack: invalid parameters or codes")
    return out


def stream_unpack(h, w, n, step, data, s_bits=5, o_bits=7):
    data = np.ascontiguousarray(data, np.uint8)
    R = n_ranges(h, w, n)
    out = dict(domain=np.zeros(R, np.int32), iso=np.zeros(R, np.uint8),
               s_idx=np.zeros(R, np.uint8), o_idx=np.zeros(R, np.uint8))
    rc = lib().oracle_stream_unpack(h, w, n, step, s_bits, o_bits, _ptr(data), len(data),
                                    _ptr(out["domain"]), _ptr(out["iso"]), _ptr(out["s_idx"]),
                                    _ptr(out["o_idx"]))
    if rc != 0:
        raise ValueError("oracle_stream_unpack: invalid stream")
    return out


def max_threads():
    return int(lib().oracle_max_threads())
