"""ctypes binding of libfic.so (argument marshalling only).

Every function here forwards to one C entry point of ``include/fic.h``; all
arithmetic runs in the library's HIP kernels.  If the library is missing this
module raises: there is no CPU fallback.
"""
import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfic.so")
# launch shapes measured by the autotuner; loaded with the library if present
TUNING_PATH = os.path.join(HERE, "tuning.json")

METHOD_MFMA = 0
METHOD_DIRECT = 1
METHOD_MFMA_I8 = 2   # 12-bit images, 8x8 ranges: the int8 matrix cores

_STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported parameters",
           3: "workspace too small", 4: "HIP runtime error"}


class FicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("bit_depth", ctypes.c_int32), ("range_size", ctypes.c_int32),
                ("domain_step", ctypes.c_int32), ("s_bits", ctypes.c_int32),
                ("o_bits", ctypes.c_int32), ("method", ctypes.c_int32),
                ("full_search", ctypes.c_int32)]


class _Codes(ctypes.Structure):
    _fields_ = [("domain", ctypes.c_void_p), ("iso", ctypes.c_void_p),
                ("s_idx", ctypes.c_void_p), ("o_idx", ctypes.c_void_p),
                ("err", ctypes.c_void_p)]


class _QtOut(ctypes.Structure):
    _fields_ = [("y", ctypes.c_void_p), ("x", ctypes.c_void_p), ("size", ctypes.c_void_p),
                ("codes", _Codes), ("n_leaves", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    """One launch-shape entry (fic_tuning of include/fic.h)."""
    _fields_ = [("bit_depth", ctypes.c_int32), ("range_size", ctypes.c_int32),
                ("method", ctypes.c_int32), ("min_domains", ctypes.c_int32),
                ("col_chunks", ctypes.c_int32), ("seed_blocks", ctypes.c_int32),
                ("item_blocks", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


@dataclass
class Params:
    height: int
    width: int
    bit_depth: int = 8
    range_size: int = 8
    domain_step: int = 4
    s_bits: int = 5
    o_bits: int = 7
    method: int = METHOD_MFMA
    full_search: int = 0   # 1: ranges and domains without variance are searched too

    def c(self):
        return _Params(self.height, self.width, self.bit_depth, self.range_size,
                       self.domain_step, self.s_bits, self.o_bits, self.method,
                       int(self.full_search))


_LIB = None


def lib():
    """Load libfic.so from the package directory (raises if it is not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1404_0774_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        P = ctypes.POINTER(_Params)
        L.fic_query.restype = ctypes.c_int
        L.fic_query.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.fic_search_counts.restype = ctypes.c_int
        L.fic_search_counts.argtypes = [P, vp, sz, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64)]
        L.fic_encode.restype = ctypes.c_int
        L.fic_encode.argtypes = [P, vp, _Codes, vp, sz, vp]
        L.fic_encode_noalloc.restype = ctypes.c_int
        L.fic_encode_noalloc.argtypes = [P, vp, _Codes, vp]
        L.fic_decode.restype = ctypes.c_int
        L.fic_decode.argtypes = [P, vp, vp, vp, vp, i32, ctypes.c_float, vp, vp]
        L.fic_decode_batch.restype = ctypes.c_int
        L.fic_decode_batch.argtypes = [P, i32, vp, vp, vp, vp, i32, ctypes.c_float, vp, vp]
        L.fic_decode_scaled.restype = ctypes.c_int
        L.fic_decode_scaled.argtypes = [P, i32, i32, vp, vp, vp, vp, i32, ctypes.c_float, vp, vp]
        L.fic_quadtree_query.restype = ctypes.c_int
        L.fic_quadtree_query.argtypes = [P, i32, ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_int64)]
        L.fic_encode_quadtree.restype = ctypes.c_int
        L.fic_encode_quadtree.argtypes = [P, i32, ctypes.c_double, vp, _QtOut, vp, sz, vp]
        L.fic_stream_query.restype = ctypes.c_int
        L.fic_stream_query.argtypes = [P, ctypes.POINTER(sz), ctypes.POINTER(i32)]
        L.fic_stream_pack.restype = ctypes.c_int
        L.fic_stream_pack.argtypes = [P, vp, vp, vp, vp, vp, sz, vp]
        L.fic_stream_header.restype = ctypes.c_int
        L.fic_stream_header.argtypes = [vp, sz, P]
        L.fic_stream_unpack.restype = ctypes.c_int
        L.fic_stream_unpack.argtypes = [P, vp, sz, vp, vp, vp, vp, vp]
        L.fic_decode_backward.restype = ctypes.c_int
        L.fic_decode_backward.argtypes = [P, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, sz, vp]
        L.fic_decode_backward_batch.restype = ctypes.c_int
        L.fic_decode_backward_batch.argtypes = [P, i32, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp,
                                                sz, vp]
        L.fic_decode_backward_batch_workspace.restype = ctypes.c_int
        L.fic_decode_backward_batch_workspace.argtypes = [P, i32, ctypes.POINTER(sz)]
        PP = ctypes.POINTER(_Params)
        L.fic_batch_query.restype = ctypes.c_int
        L.fic_batch_query.argtypes = [PP, i32, ctypes.POINTER(sz)]
        L.fic_batch_prepare.restype = ctypes.c_int
        L.fic_batch_prepare.argtypes = [PP, i32, ctypes.POINTER(vp), ctypes.POINTER(_Codes), vp, sz]
        L.fic_encode_batch.restype = ctypes.c_int
        L.fic_encode_batch.argtypes = [PP, i32, vp, sz, vp, vp]
        L.fic_refine.restype = ctypes.c_int
        L.fic_refine.argtypes = [P, vp, vp, vp, vp, vp, i32, ctypes.c_float, i32, ctypes.c_float,
                                 ctypes.c_float, vp, vp, sz, vp]
        L.fic_refine_workspace.restype = ctypes.c_int
        L.fic_refine_workspace.argtypes = [P, i32, ctypes.POINTER(sz)]
        L.fic_timing_begin.restype = ctypes.c_int
        L.fic_timing_begin.argtypes = []
        L.fic_timing_end.restype = ctypes.c_int
        L.fic_timing_end.argtypes = [ctypes.POINTER(ctypes.c_int32)] + [ctypes.POINTER(ctypes.c_double)] * 4
        TP = ctypes.POINTER(Tuning)
        L.fic_set_tuning.restype = ctypes.c_int
        L.fic_set_tuning.argtypes = [TP, i32]
        L.fic_load_tuning.restype = ctypes.c_int
        L.fic_load_tuning.argtypes = [ctypes.c_char_p]
        L.fic_get_tuning.restype = ctypes.c_int
        L.fic_get_tuning.argtypes = [P, TP]
        L.fic_status_string.restype = ctypes.c_char_p
        L.fic_status_string.argtypes = [ctypes.c_int]
        L.fic_last_error.restype = ctypes.c_char_p
        L.fic_last_error.argtypes = []
        _LIB = L
        if os.path.exists(TUNING_PATH):
            _check(L.fic_load_tuning(TUNING_PATH.encode()))
    return _LIB


def set_tuning(entries):
    """Replace the launch-shape table; entries are dicts with Tuning's fields
    (missing col_chunks / item_blocks = 0 and seed_blocks = -1: defaults)."""
    arr = (Tuning * max(1, len(entries)))()
    for i, e in enumerate(entries):
        arr[i] = Tuning(e["bit_depth"], e["range_size"], e["method"], e.get("min_domains", 0),
                        e.get("col_chunks", 0), e.get("seed_blocks", -1), e.get("item_blocks", 0))
    _check(lib().fic_set_tuning(arr, len(entries)))


def load_tuning(path):
    """Replace the launch-shape table with the entries of a JSON file."""
    _check(lib().fic_load_tuning(os.fsencode(path)))


def get_tuning(p: "Params"):
    """The launch shape fic_encode resolves for these parameters (dict)."""
    t = Tuning()
    cp = p.c()
    _check(lib().fic_get_tuning(ctypes.byref(cp), ctypes.byref(t)))
    return t.as_dict()


def _check(status):
    if status != 0:
        raise FicError(status, lib().fic_last_error().decode())


def query(p: Params):
    """Host-only: (n_ranges, n_domains, encode_ws_bytes, backward_ws_bytes)."""
    nr, nd = ctypes.c_int64(), ctypes.c_int64()
    ew, bw = ctypes.c_size_t(), ctypes.c_size_t()
    cp = p.c()
    _check(lib().fic_query(ctypes.byref(cp), ctypes.byref(nr), ctypes.byref(nd),
                           ctypes.byref(ew), ctypes.byref(bw)))
    return nr.value, nd.value, ew.value, bw.value


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(nbytes, device):
    # 256-byte aligned view into a torch allocation
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


def _dev_ptr(t, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def encode(image: torch.Tensor, p: Params, workspace=None):
    """Encode one image (device tensor, uint8 or int16/uint16 holding 12-bit
    values).  Returns a dict of device tensors: domain (int32), iso (uint8),
    s_idx (uint8), o_idx (uint8), err (float64)."""
    exp = torch.uint8 if p.bit_depth == 8 else torch.uint16
    if image.dtype == torch.int16 and p.bit_depth == 12:
        image = image.view(torch.uint16)
    img_ptr = _dev_ptr(image, exp, "image")
    if tuple(image.shape) != (p.height, p.width):
        raise ValueError(f"image shape {tuple(image.shape)} != {(p.height, p.width)}")
    nr, nd, ew, _ = query(p)
    dev = image.device
    out = dict(domain=torch.empty(nr, dtype=torch.int32, device=dev),
               iso=torch.empty(nr, dtype=torch.uint8, device=dev),
               s_idx=torch.empty(nr, dtype=torch.uint8, device=dev),
               o_idx=torch.empty(nr, dtype=torch.uint8, device=dev),
               err=torch.empty(nr, dtype=torch.float64, device=dev))
    if workspace is None:
        keep, ws = _workspace(ew, dev)
    else:
        keep, ws = workspace, workspace.data_ptr()
        if workspace.numel() * workspace.element_size() < ew:
            raise ValueError("workspace too small")
    codes = _Codes(out["domain"].data_ptr(), out["iso"].data_ptr(), out["s_idx"].data_ptr(),
                   out["o_idx"].data_ptr(), out["err"].data_ptr())
    cp = p.c()
    _check(lib().fic_encode(ctypes.byref(cp), ctypes.c_void_p(img_ptr), codes,
                            ctypes.c_void_p(ws), ctypes.c_size_t(ew), _stream(dev)))
    out["_ws"] = keep
    out["_ws_ptr"] = (ws, ew)
    return out


def quadtree_query(p: Params, min_range_size: int):
    """Host-only: (workspace bytes, largest leaf count)."""
    nb, ml = ctypes.c_size_t(), ctypes.c_int64()
    cp = p.c()
    _check(lib().fic_quadtree_query(ctypes.byref(cp), min_range_size, ctypes.byref(nb),
                                    ctypes.byref(ml)))
    return nb.value, ml.value


def encode_quadtree(image: torch.Tensor, p: Params, min_range_size: int, tau: float):
    """Quadtree encode: ranges of side p.range_size whose residual exceeds
    tau * n^2 are split into quadrants down to min_range_size.  Returns a
    dict of device leaf arrays (y, x, size, domain, iso, s_idx, o_idx, err)
    trimmed to the leaf count (this synchronises the device)."""
    exp = torch.uint8 if p.bit_depth == 8 else torch.uint16
    if image.dtype == torch.int16 and p.bit_depth == 12:
        image = image.view(torch.uint16)
    img_ptr = _dev_ptr(image, exp, "image")
    wsb, ml = quadtree_query(p, min_range_size)
    dev = image.device
    out = dict(y=torch.empty(ml, dtype=torch.int32, device=dev),
               x=torch.empty(ml, dtype=torch.int32, device=dev),
               size=torch.empty(ml, dtype=torch.uint8, device=dev),
               domain=torch.empty(ml, dtype=torch.int32, device=dev),
               iso=torch.empty(ml, dtype=torch.uint8, device=dev),
               s_idx=torch.empty(ml, dtype=torch.uint8, device=dev),
               o_idx=torch.empty(ml, dtype=torch.uint8, device=dev),
               err=torch.empty(ml, dtype=torch.float64, device=dev))
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    keep, ws = _workspace(wsb, dev)
    q = _QtOut(out["y"].data_ptr(), out["x"].data_ptr(), out["size"].data_ptr(),
               _Codes(out["domain"].data_ptr(), out["iso"].data_ptr(), out["s_idx"].data_ptr(),
                      out["o_idx"].data_ptr(), out["err"].data_ptr()), count.data_ptr())
    cp = p.c()
    _check(lib().fic_encode_quadtree(ctypes.byref(cp), min_range_size, ctypes.c_double(tau),
                                     ctypes.c_void_p(img_ptr), q, ctypes.c_void_p(ws),
                                     ctypes.c_size_t(wsb), _stream(dev)))
    n = int(count.item())
    del keep
    return {k: v[:n] for k, v in out.items()}


def search_counts(out, p: Params):
    """(ranges, domains) the search kernel visited in the encode that
    produced `out`; it evaluated 8 * ranges * domains candidates.
    Synchronises the device."""
    ws, ew = out["_ws_ptr"]
    nr, nd = ctypes.c_int64(), ctypes.c_int64()
    cp = p.c()
    _check(lib().fic_search_counts(ctypes.byref(cp), ctypes.c_void_p(ws), ctypes.c_size_t(ew),
                                   ctypes.byref(nr), ctypes.byref(nd)))
    return nr.value, nd.value


class Batch:
    """A prepared batch of slices (device images, codes and workspace kept
    alive here).  run() enqueues fic_encode_batch on the current stream."""

    def __init__(self, images, params):
        if len(images) != len(params) or not images:
            raise ValueError("need one Params per image")
        self.params = list(params)
        n = len(images)
        self._cp = (_Params * n)(*[p.c() for p in params])
        nbytes = ctypes.c_size_t()
        _check(lib().fic_batch_query(self._cp, n, ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        dev = images[0].device
        self._keep, self._ws = _workspace(self.ws_bytes, dev)
        self.images = []
        self.codes = []
        for img, p in zip(images, params):
            exp = torch.uint8 if p.bit_depth == 8 else torch.uint16
            if img.dtype == torch.int16 and p.bit_depth == 12:
                img = img.view(torch.uint16)
            _dev_ptr(img, exp, "image")
            if tuple(img.shape) != (p.height, p.width):
                raise ValueError("image shape does not match its Params")
            nr = (p.height // p.range_size) * (p.width // p.range_size)
            self.images.append(img)
            self.codes.append(dict(domain=torch.empty(nr, dtype=torch.int32, device=dev),
                                   iso=torch.empty(nr, dtype=torch.uint8, device=dev),
                                   s_idx=torch.empty(nr, dtype=torch.uint8, device=dev),
                                   o_idx=torch.empty(nr, dtype=torch.uint8, device=dev),
                                   err=torch.empty(nr, dtype=torch.float64, device=dev)))
        self.ticks = torch.zeros(n + 1, dtype=torch.int64, device=dev)
        ptrs = (ctypes.c_void_p * n)(*[im.data_ptr() for im in self.images])
        outs = (_Codes * n)(*[_Codes(c["domain"].data_ptr(), c["iso"].data_ptr(),
                                     c["s_idx"].data_ptr(), c["o_idx"].data_ptr(),
                                     c["err"].data_ptr()) for c in self.codes])
        _check(lib().fic_batch_prepare(self._cp, n, ptrs, outs, ctypes.c_void_p(self._ws),
                                       ctypes.c_size_t(self.ws_bytes)))

    def run(self):
        dev = self.images[0].device
        _check(lib().fic_encode_batch(self._cp, len(self.images), ctypes.c_void_p(self._ws),
                                      ctypes.c_size_t(self.ws_bytes),
                                      ctypes.c_void_p(self.ticks.data_ptr()), _stream(dev)))
        return self.codes


def stream_query(p: Params):
    """Host-only: (stream bytes, bits per range record)."""
    nb, rb = ctypes.c_size_t(), ctypes.c_int32()
    cp = p.c()
    _check(lib().fic_stream_query(ctypes.byref(cp), ctypes.byref(nb), ctypes.byref(rb)))
    return nb.value, rb.value


def stream_pack(codes, p: Params):
    """The code stream of device codes (dict with domain, iso, s_idx, o_idx)
    as a device uint8 tensor."""
    nb, _ = stream_query(p)
    dev = codes["domain"].device
    out = torch.empty((nb + 3) // 4, dtype=torch.int32, device=dev)
    cp = p.c()
    _check(lib().fic_stream_pack(ctypes.byref(cp), _dev_ptr(codes["domain"], torch.int32, "domain"),
                                 _dev_ptr(codes["iso"], torch.uint8, "iso"),
                                 _dev_ptr(codes["s_idx"], torch.uint8, "s_idx"),
                                 _dev_ptr(codes["o_idx"], torch.uint8, "o_idx"),
                                 out.data_ptr(), nb, _stream(dev)))
    return out.view(torch.uint8)[:nb]


def stream_header(data) -> Params:
    """Params of a stream from its first 32 bytes (bytes or a host array)."""
    buf = bytes(memoryview(data)[:32]) if not isinstance(data, torch.Tensor) else \
        bytes(data[:32].cpu().numpy().tobytes())
    q = _Params()
    _check(lib().fic_stream_header(ctypes.c_char_p(buf), len(buf), ctypes.byref(q)))
    return Params(q.height, q.width, q.bit_depth, q.range_size, q.domain_step, q.s_bits,
                  q.o_bits, q.method, q.full_search)


def stream_unpack(data: torch.Tensor, p: Params = None):
    """Codes (device dict: domain, iso, s_idx, o_idx) of a device stream."""
    if p is None:
        p = stream_header(data)
    nr = query(p)[0]
    dev = data.device
    buf = data
    if buf.data_ptr() % 4:
        buf = buf.clone()
    out = dict(domain=torch.empty(nr, dtype=torch.int32, device=dev),
               iso=torch.empty(nr, dtype=torch.uint8, device=dev),
               s_idx=torch.empty(nr, dtype=torch.uint8, device=dev),
               o_idx=torch.empty(nr, dtype=torch.uint8, device=dev))
    cp = p.c()
    _check(lib().fic_stream_unpack(ctypes.byref(cp), _dev_ptr(buf, torch.uint8, "stream"),
                                   buf.numel(), out["domain"].data_ptr(), out["iso"].data_ptr(),
                                   out["s_idx"].data_ptr(), out["o_idx"].data_ptr(), _stream(dev)))
    return out


def dequantize(s_idx, o_idx, p: Params):
    """Grid values of quantised codes: s = s_idx/2^(s_bits-1) - 1, o = o_idx*delta_o - 2^bits."""
    s = s_idx.to(torch.float32) / float(2 ** (p.s_bits - 1)) - 1.0
    P = float(2 ** p.bit_depth)
    o = o_idx.to(torch.float32) * (2.0 * P / 2 ** p.o_bits) - P
    return s, o


def decode(domain, iso, s, o, p: Params, iters=12, x0=None):
    """Iterate the PIFS map; returns the trajectory (iters+1, H, W) float32."""
    if x0 is None:
        x0 = float(2 ** (p.bit_depth - 1))
    dev = s.device
    traj = torch.empty((iters + 1, p.height, p.width), dtype=torch.float32, device=dev)
    cp = p.c()
    _check(lib().fic_decode(ctypes.byref(cp), _dev_ptr(domain, torch.int32, "domain"),
                            _dev_ptr(iso, torch.uint8, "iso"), _dev_ptr(s, torch.float32, "s"),
                            _dev_ptr(o, torch.float32, "o"), iters, ctypes.c_float(x0),
                            traj.data_ptr(), _stream(dev)))
    return traj


def decode_batch(domain, iso, s, o, p: Params, iters=12, x0=None):
    """Decode B images of one geometry, each with its own codes (tensors of
    shape (B, n_ranges)); returns the trajectories (B, iters+1, H, W)."""
    if x0 is None:
        x0 = float(2 ** (p.bit_depth - 1))
    B = domain.shape[0]
    dev = s.device
    traj = torch.empty((B, iters + 1, p.height, p.width), dtype=torch.float32, device=dev)
    cp = p.c()
    _check(lib().fic_decode_batch(ctypes.byref(cp), B, _dev_ptr(domain, torch.int32, "domain"),
                                  _dev_ptr(iso, torch.uint8, "iso"), _dev_ptr(s, torch.float32, "s"),
                                  _dev_ptr(o, torch.float32, "o"), iters, ctypes.c_float(x0),
                                  traj.data_ptr(), _stream(dev)))
    return traj


def decode_scaled(domain, iso, s, o, p: Params, scale=(2, 1), iters=12, x0=None):
    """Decode codes of the image described by p at scale num/den; returns the
    trajectory (iters+1, H*num/den, W*num/den) float32."""
    num, den = scale
    if x0 is None:
        x0 = float(2 ** (p.bit_depth - 1))
    if (p.height * num) % den or (p.width * num) % den:
        raise ValueError("the scaled image is not whole pixels")
    dev = s.device
    traj = torch.empty((iters + 1, p.height * num // den, p.width * num // den),
                       dtype=torch.float32, device=dev)
    cp = p.c()
    _check(lib().fic_decode_scaled(ctypes.byref(cp), num, den,
                                   _dev_ptr(domain, torch.int32, "domain"),
                                   _dev_ptr(iso, torch.uint8, "iso"),
                                   _dev_ptr(s, torch.float32, "s"), _dev_ptr(o, torch.float32, "o"),
                                   iters, ctypes.c_float(x0), traj.data_ptr(), _stream(dev)))
    return traj


def decode_backward(domain, iso, s, o, traj, grad_xT, p: Params):
    """dL/ds, dL/do of the unrolled decoder given dL/dx_T."""
    iters = traj.shape[0] - 1
    dev = s.device
    nr, _, _, bw = query(p)
    gs = torch.empty(nr, dtype=torch.float32, device=dev)
    go = torch.empty(nr, dtype=torch.float32, device=dev)
    keep, ws = _workspace(bw, dev)
    cp = p.c()
    g = grad_xT.contiguous()
    _check(lib().fic_decode_backward(ctypes.byref(cp), _dev_ptr(domain, torch.int32, "domain"),
                                     _dev_ptr(iso, torch.uint8, "iso"),
                                     _dev_ptr(s, torch.float32, "s"), _dev_ptr(o, torch.float32, "o"),
                                     iters, _dev_ptr(traj, torch.float32, "traj"),
                                     _dev_ptr(g, torch.float32, "grad_xT"), gs.data_ptr(),
                                     go.data_ptr(), ctypes.c_void_p(ws), ctypes.c_size_t(bw),
                                     _stream(dev)))
    del keep
    return gs, go


def decode_backward_batch(domain, iso, s, o, traj, grad_xT, p: Params):
    """dL/ds, dL/do of B decoders of one geometry (codes (B, n_ranges), traj
    (B, iters+1, H, W) as decode_batch returns, grad_xT (B, H, W)); returns
    two (B, n_ranges) tensors."""
    B = domain.shape[0]
    iters = traj.shape[1] - 1
    dev = s.device
    nr = query(p)[0]
    cp = p.c()
    nbytes = ctypes.c_size_t()
    _check(lib().fic_decode_backward_batch_workspace(ctypes.byref(cp), B, ctypes.byref(nbytes)))
    gs = torch.empty((B, nr), dtype=torch.float32, device=dev)
    go = torch.empty((B, nr), dtype=torch.float32, device=dev)
    keep, ws = _workspace(nbytes.value, dev)
    g = grad_xT.contiguous()
    _check(lib().fic_decode_backward_batch(
        ctypes.byref(cp), B, _dev_ptr(domain, torch.int32, "domain"),
        _dev_ptr(iso, torch.uint8, "iso"), _dev_ptr(s, torch.float32, "s"),
        _dev_ptr(o, torch.float32, "o"), iters, _dev_ptr(traj, torch.float32, "traj"),
        _dev_ptr(g, torch.float32, "grad_xT"), gs.data_ptr(), go.data_ptr(),
        ctypes.c_void_p(ws), nbytes, _stream(dev)))
    del keep
    return gs, go


def refine(domain, iso, s, o, image, p: Params, iters=12, steps=50, lr_s=5e-3, lr_o=0.5,
           x0=None):
    """Adam refinement of (s, o) against the decoded attractor's error, indices
    fixed.  s and o (float32 device tensors) are updated in place; returns the
    loss before each step and after the last (float64 device tensor)."""
    if x0 is None:
        x0 = float(2 ** (p.bit_depth - 1))
    dev = s.device
    exp = torch.uint8 if p.bit_depth == 8 else torch.uint16
    if image.dtype == torch.int16 and p.bit_depth == 12:
        image = image.view(torch.uint16)
    nbytes = ctypes.c_size_t()
    cp = p.c()
    _check(lib().fic_refine_workspace(ctypes.byref(cp), iters, ctypes.byref(nbytes)))
    keep, ws = _workspace(nbytes.value, dev)
    loss = torch.empty(steps + 1, dtype=torch.float64, device=dev)
    _check(lib().fic_refine(ctypes.byref(cp), _dev_ptr(domain, torch.int32, "domain"),
                            _dev_ptr(iso, torch.uint8, "iso"), _dev_ptr(s, torch.float32, "s"),
                            _dev_ptr(o, torch.float32, "o"), _dev_ptr(image, exp, "image"), iters,
                            ctypes.c_float(x0), steps, ctypes.c_float(lr_s), ctypes.c_float(lr_o),
                            loss.data_ptr(), ctypes.c_void_p(ws), ctypes.c_size_t(nbytes.value),
                            _stream(dev)))
    loss._ws = keep
    return loss


def timing_begin():
    """Start per-phase event timing of fic_encode calls (benchmark support)."""
    _check(lib().fic_timing_begin())


def timing_end():
    """Stop timing; returns (n_calls, ms_prep, ms_seed, ms_search, ms_finalize)
    summed over the timed calls."""
    n = ctypes.c_int32()
    v = [ctypes.c_double() for _ in range(4)]
    _check(lib().fic_timing_end(ctypes.byref(n), *[ctypes.byref(x) for x in v]))
    return (n.value,) + tuple(x.value for x in v)


class FicDecode(torch.autograd.Function):
    """x_T = decode(s, o) with domain and transform indices held fixed; the
    backward pass is the library's hand-written adjoint."""

    @staticmethod
    def forward(ctx, s, o, domain, iso, p, iters, x0):
        s = s.contiguous()
        o = o.contiguous()
        traj = decode(domain, iso, s, o, p, iters, x0)
        ctx.save_for_backward(s, o, domain, iso, traj)
        ctx.p = p
        return traj[-1]

    @staticmethod
    def backward(ctx, g):
        s, o, domain, iso, traj = ctx.saved_tensors
        gs, go = decode_backward(domain, iso, s, o, traj, g.contiguous(), ctx.p)
        return gs, go, None, None, None, None, None
