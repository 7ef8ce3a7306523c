"""Host-side checks of the C ABI: the library loads without a GPU, exports
every entry point declared in include/fic.h, and rejects bad arguments with
the documented status codes before touching the GPU."""
import ctypes
import os
import re

import pytest

import paper_1404_0774_amd as F
from paper_1404_0774_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(fic_\w+)\s*\(", src, flags=re.M)
    return names


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert {"fic_query", "fic_encode", "fic_decode", "fic_decode_backward",
            "fic_status_string", "fic_last_error"} <= set(names)
    L = F.lib()
    for n in names:
        assert hasattr(L, n), n


def test_query_counts_and_workspace():
    nr, nd, ew, bw = F.query(F.Params(512, 512, 8, 8, 4))
    assert (nr, nd) == (4096, 15625)
    assert ew > 15625 * 64 * 2 + 4096 * 8 * 64 * 2 and bw > 0
    nr, nd, _, _ = F.query(F.Params(64, 64, 8, 4, 4))
    assert (nr, nd) == (256, 225)
    nr, nd, _, _ = F.query(F.Params(256, 256, 8, 4, 4))
    assert (nr, nd) == (4096, 63 * 63)
    nr, nd, _, _ = F.query(F.Params(512, 512, 12, 8, 2))
    assert (nr, nd) == (4096, 249 * 249)


@pytest.mark.parametrize("kw,status", [
    (dict(height=500), 1), (dict(width=0), 1), (dict(domain_step=0), 1),
    (dict(range_size=3, height=63, width=63), 2), (dict(bit_depth=10), 2),
    (dict(s_bits=0), 2), (dict(s_bits=9), 2), (dict(o_bits=10), 2),
    (dict(height=8, width=8), 1),
])
def test_query_rejects(kw, status):
    base = dict(height=512, width=512, bit_depth=8, range_size=8, domain_step=4)
    base.update(kw)
    with pytest.raises(F.FicError) as e:
        F.query(F.Params(**base))
    assert e.value.status == status
    assert F.lib().fic_last_error().decode() != ""


def test_too_many_candidates_rejected():
    # 12-bit keys keep 19 candidate bits: a 2048^2 image at stride 1 is beyond them
    with pytest.raises(F.FicError) as e:
        F.query(F.Params(2048, 2048, 12, 8, 1))
    assert e.value.status == 2


def test_encode_validates_before_gpu_work():
    L = F.lib()
    p = F.Params(64, 64, 8, 4, 4).c()
    codes = _lib._Codes(0, 0, 0, 0, 0)
    st = L.fic_encode(ctypes.byref(p), None, codes, None, 0, None)
    assert st == 1 and b"null" in L.fic_last_error()
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: validation fails first
    codes = _lib._Codes(fake, fake, fake, fake, fake)
    st = L.fic_encode(ctypes.byref(p), fake, codes, ctypes.c_void_p((1 << 20) + 8), 1 << 30, None)
    assert st == 1 and b"aligned" in L.fic_last_error()
    st = L.fic_encode(ctypes.byref(p), fake, codes, fake, 16, None)
    assert st == 3
    bad = F.Params(64, 64, 8, 4, 4, method=7).c()
    assert L.fic_encode(ctypes.byref(bad), fake, codes, fake, 1 << 30, None) == 1
    assert L.fic_encode(None, fake, codes, fake, 1 << 30, None) == 1


def test_decode_validates_before_gpu_work():
    L = F.lib()
    p = F.Params(64, 64, 8, 4, 4).c()
    fake = ctypes.c_void_p(1 << 20)
    assert L.fic_decode(ctypes.byref(p), None, fake, fake, fake, 12, ctypes.c_float(128), fake, None) == 1
    assert L.fic_decode(ctypes.byref(p), fake, fake, fake, fake, -1, ctypes.c_float(128), fake, None) == 1
    assert L.fic_decode_backward(ctypes.byref(p), fake, fake, fake, fake, 12, fake, fake, fake,
                                 fake, fake, 0, None) == 3


def test_status_strings():
    L = F.lib()
    for s in range(5):
        assert L.fic_status_string(s)
    assert L.fic_status_string(99) == b"unknown status"
