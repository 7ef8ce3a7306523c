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
