"""Host-side checks of the C ABI: the library loads without a GPU, exports
every entry point declared in include/fic.h, and rejects bad arguments with
the documented status codes before touching the GPU."""
import ctypes

import numpy as np
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
    assert {"fic_query", "fic_encode", "fic_decode", "fic_decode_backward", "fic_refine",
            "fic_refine_workspace", "fic_timing_begin", "fic_timing_end",
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
    (dict(bit_depth=12, o_bits=9), 2),   # offset indices are one byte
    (dict(height=8, width=8), 1), (dict(full_search=2), 1), (dict(full_search=-1), 1),
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


def test_backward_batch_validates_before_gpu_work():
    L = F.lib()
    p = F.Params(64, 64, 8, 4, 4).c()
    fake = ctypes.c_void_p(1 << 20)
    one, four = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.fic_decode_backward_batch_workspace(ctypes.byref(p), 1, ctypes.byref(one)) == 0
    assert L.fic_decode_backward_batch_workspace(ctypes.byref(p), 4, ctypes.byref(four)) == 0
    assert four.value == 4 * one.value and one.value % 256 == 0
    assert L.fic_decode_backward_batch_workspace(ctypes.byref(p), 0, ctypes.byref(one)) == 1
    args = lambda n, ws_bytes: [ctypes.byref(p), n, fake, fake, fake, fake, 12, fake, fake, fake,
                                fake, fake, ws_bytes, None]
    assert L.fic_decode_backward_batch(*args(0, four.value)) == 1          # no images
    assert L.fic_decode_backward_batch(*args(4, four.value - 1)) == 3      # workspace
    assert L.fic_decode_backward_batch(*args(70000, 1 << 40)) == 2         # > 65535 images
    big = F.Params(264, 272, 8, 4, 1).c()                                  # 68,105 domains
    assert L.fic_decode_backward_batch(ctypes.byref(big), 2, fake, fake, fake, fake, 12, fake,
                                       fake, fake, fake, fake, 1 << 40, None) == 2


def test_refine_validates_before_gpu_work():
    L = F.lib()
    p = F.Params(64, 64, 8, 4, 4).c()
    fake = ctypes.c_void_p(1 << 20)
    nbytes = ctypes.c_size_t()
    assert L.fic_refine_workspace(ctypes.byref(p), 12, ctypes.byref(nbytes)) == 0
    assert nbytes.value >= 13 * 64 * 64 * 4
    assert L.fic_refine_workspace(ctypes.byref(p), -1, ctypes.byref(nbytes)) == 1
    args = [fake, fake, fake, fake, fake, 12, ctypes.c_float(128), 50, ctypes.c_float(5e-3),
            ctypes.c_float(0.5), fake, fake, nbytes.value, None]
    bad = list(args); bad[0] = None
    assert L.fic_refine(ctypes.byref(p), *bad) == 1
    bad = list(args); bad[7] = -1
    assert L.fic_refine(ctypes.byref(p), *bad) == 1
    bad = list(args); bad[8] = ctypes.c_float(-1.0)
    assert L.fic_refine(ctypes.byref(p), *bad) == 1
    bad = list(args); bad[12] = 16
    assert L.fic_refine(ctypes.byref(p), *bad) == 3


def test_status_strings():
    L = F.lib()
    for s in range(5):
        assert L.fic_status_string(s)
    assert L.fic_status_string(99) == b"unknown status"


def test_batch_query_validation():
    L = F.lib()
    P = _lib._Params
    nbytes = ctypes.c_size_t()
    ok = (P * 2)(F.Params(64, 64, 8, 8, 8).c(), F.Params(128, 96, 8, 8, 4).c())
    assert L.fic_batch_query(ok, 2, ctypes.byref(nbytes)) == 0 and nbytes.value > 0
    mixed = (P * 2)(F.Params(64, 64, 8, 8, 8).c(), F.Params(64, 64, 8, 4, 8).c())
    assert L.fic_batch_query(mixed, 2, ctypes.byref(nbytes)) == 1
    twelve = (P * 1)(F.Params(64, 64, 12, 8, 8).c())
    assert L.fic_batch_query(twelve, 1, ctypes.byref(nbytes)) == 2
    assert L.fic_batch_query(ok, 0, ctypes.byref(nbytes)) == 1
    bad = (P * 1)(F.Params(60, 64, 8, 8, 8).c())
    assert L.fic_batch_query(bad, 1, ctypes.byref(nbytes)) == 1
    fake = ctypes.c_void_p(1 << 20)
    assert L.fic_encode_batch(ok, 2, fake, 16, None, None) in (1, 3)


@pytest.fixture
def clean_tuning():
    """Run with an empty launch-shape table; restore the shipped one after."""
    F.set_tuning([])
    yield
    if os.path.exists(_lib.TUNING_PATH):
        F.load_tuning(_lib.TUNING_PATH)
    else:
        F.set_tuning([])


def test_tuning_defaults(clean_tuning):
    # 512x512, n = 8, STEP 4: 4096 ranges = 64 row groups, 15,625 domains in
    # 489 column blocks -> about two workgroups per CU (512 / 64 = 8 chunks)
    # (the 8-bit, n = 8 matrix-core search seeds itself: no seed pass)
    t = F.get_tuning(F.Params(512, 512, 8, 8, 4))
    assert t == dict(bit_depth=8, range_size=8, method=0, min_domains=15625,
                     col_chunks=8, seed_blocks=0, item_blocks=16)
    td = F.get_tuning(F.Params(512, 512, 8, 8, 4, method=F.METHOD_DIRECT))
    assert td["seed_blocks"] == 1
    # 12-bit matrix-core searches use 16-range row groups and about 24
    # workgroups per CU: 256 groups -> 6144 / 256 = 24 chunks
    t12 = F.get_tuning(F.Params(512, 512, 12, 8, 2))
    assert t12["col_chunks"] == 24 and t12["seed_blocks"] == 1
    # fewer than 16 column blocks: no seed pass; chunks clamped to the blocks
    t1 = F.get_tuning(F.Params(64, 64, 8, 4, 4))   # 225 domains -> 8 blocks
    assert t1["seed_blocks"] == 0 and t1["col_chunks"] == 8


def test_tuning_table_selection(clean_tuning):
    p = F.Params(512, 512, 8, 8, 4)
    F.set_tuning([dict(bit_depth=8, range_size=8, method=0, min_domains=0, col_chunks=4),
                  dict(bit_depth=8, range_size=8, method=0, min_domains=10000, col_chunks=12,
                       seed_blocks=2, item_blocks=8),
                  dict(bit_depth=8, range_size=8, method=0, min_domains=20000, col_chunks=3),
                  dict(bit_depth=8, range_size=8, method=1, min_domains=0, col_chunks=5)])
    t = F.get_tuning(p)
    # the self-seeding 8-bit, n = 8 matrix-core search ignores seed_blocks
    assert (t["col_chunks"], t["seed_blocks"], t["item_blocks"]) == (12, 0, 8)
    p12 = F.Params(512, 512, 12, 8, 4)
    F.set_tuning([dict(bit_depth=12, range_size=8, method=0, min_domains=0, seed_blocks=3)])
    assert F.get_tuning(p12)["seed_blocks"] == 3
    F.set_tuning([dict(bit_depth=8, range_size=8, method=0, min_domains=0, col_chunks=4),
                  dict(bit_depth=8, range_size=8, method=0, min_domains=10000, col_chunks=12,
                       seed_blocks=2, item_blocks=8),
                  dict(bit_depth=8, range_size=8, method=0, min_domains=20000, col_chunks=3),
                  dict(bit_depth=8, range_size=8, method=1, min_domains=0, col_chunks=5)])
    p.method = F.METHOD_DIRECT
    t = F.get_tuning(p)
    assert (t["col_chunks"], t["seed_blocks"], t["item_blocks"]) == (5, 1, 16)
    small = F.Params(128, 128, 8, 8, 4)              # 841 domains: first entry
    assert F.get_tuning(small)["col_chunks"] == 4
    # clamping: seed and chunks at most the block count
    F.set_tuning([dict(bit_depth=8, range_size=4, method=0, col_chunks=4096, seed_blocks=64)])
    t = F.get_tuning(F.Params(64, 64, 8, 4, 4))      # 8 column blocks
    assert t["seed_blocks"] == 8 and t["col_chunks"] == 8
    F.set_tuning([])
    assert F.get_tuning(F.Params(512, 512, 8, 8, 4))["col_chunks"] == 8


@pytest.mark.parametrize("field,value", [("bit_depth", 10), ("range_size", 6), ("method", 3),
                                         ("min_domains", -1), ("col_chunks", -1),
                                         ("col_chunks", 5000), ("seed_blocks", -2),
                                         ("seed_blocks", 65), ("item_blocks", -3)])
def test_tuning_rejects_bad_entries(clean_tuning, field, value):
    F.set_tuning([dict(bit_depth=8, range_size=8, method=0, col_chunks=6)])
    e = dict(bit_depth=8, range_size=8, method=0)
    e[field] = value
    with pytest.raises(F.FicError) as ex:
        F.set_tuning([e])
    assert ex.value.status == 1
    # the table is unchanged after a rejected call
    assert F.get_tuning(F.Params(512, 512, 8, 8, 4))["col_chunks"] == 6


def test_tuning_json(clean_tuning, tmp_path):
    good = tmp_path / "t.json"
    good.write_text('{"device": "any", "entries": [\n'
                    ' {"bit_depth": 8, "range_size": 8, "method": 0, "min_domains": 0,\n'
                    '  "col_chunks": 6, "seed_blocks": 2, "item_blocks": 32, "ms": 0.16,\n'
                    '  "sweep": [1, 2, {"x": null}], "ok": true}\n], "note": "a \\"quoted\\" word"}')
    F.load_tuning(str(good))
    t = F.get_tuning(F.Params(512, 512, 8, 8, 4, method=F.METHOD_MFMA))
    assert (t["col_chunks"], t["seed_blocks"], t["item_blocks"]) == (6, 0, 32)
    t4 = F.get_tuning(F.Params(512, 512, 8, 4, 4))   # n = 4: no entry, defaults
    assert t4["seed_blocks"] == 1 and t4["item_blocks"] == 16
    for bad in ['{"entries": [{"bit_depth": 8, "range_size": 8, "method": 0,}]}',
                '{"entries": [{"bit_depth": 8, "range_size": 8, "method": 0, "col_chunks": 1.5}]}',
                '{"entries": [{"bit_depth": 9, "range_size": 8, "method": 0}]}',
                '{"entries": [', '[] x']:
        f = tmp_path / "bad.json"
        f.write_text(bad)
        with pytest.raises(F.FicError):
            F.load_tuning(str(f))
        assert F.get_tuning(F.Params(512, 512, 8, 8, 4))["col_chunks"] == 6
    with pytest.raises(F.FicError):
        F.load_tuning(str(tmp_path / "missing.json"))


def test_search_counts_validation():
    L = F.lib()
    p = F.Params(64, 64, 8, 8, 4).c()
    nr, nd = ctypes.c_int64(), ctypes.c_int64()
    fake = ctypes.c_void_p(1 << 20)
    ws = F.query(F.Params(64, 64, 8, 8, 4))[2]
    assert L.fic_search_counts(ctypes.byref(p), None, ws, ctypes.byref(nr), ctypes.byref(nd)) == 1
    assert L.fic_search_counts(ctypes.byref(p), fake, ws, None, ctypes.byref(nd)) == 1
    assert L.fic_search_counts(ctypes.byref(p), fake, 16, ctypes.byref(nr), ctypes.byref(nd)) == 1
    pd = F.Params(64, 64, 8, 8, 4, method=F.METHOD_DIRECT, full_search=3).c()
    assert L.fic_search_counts(ctypes.byref(pd), fake, ws, ctypes.byref(nr), ctypes.byref(nd)) == 1
    p12 = F.Params(64, 64, 12, 8, 4).c()  # 12-bit: validated like 8-bit
    assert L.fic_search_counts(ctypes.byref(p12), fake, 16, ctypes.byref(nr), ctypes.byref(nd)) == 1


@pytest.mark.parametrize("H,W,bits,n,step,sb,ob", [(64, 64, 8, 4, 4, 5, 7), (512, 512, 8, 8, 4, 5, 7),
                                                   (512, 512, 12, 8, 2, 5, 7), (40, 56, 8, 4, 3, 3, 6)])
def test_stream_query_and_header_match_the_oracle_format(H, W, bits, n, step, sb, ob):
    """The library's stream size and header parsing agree with the oracle's
    writer of the same format (host only)."""
    from oracle import oracle as O
    p = F.Params(H, W, bits, n, step, s_bits=sb, o_bits=ob)
    nb, B = F.stream_query(p)
    assert nb == O.stream_bytes(H, W, n, step, sb, ob)
    assert B == O.stream_domain_bits(O.n_domains(H, W, n, step)) + 3 + sb + ob
    R = (H // n) * (W // n)
    zero = dict(domain=np.zeros(R, np.int32), iso=np.zeros(R, np.uint8),
                s_idx=np.zeros(R, np.uint8), o_idx=np.zeros(R, np.uint8))
    data = O.stream_pack(H, W, n, step, zero, bits=bits, s_bits=sb, o_bits=ob)
    q = F.stream_header(data.tobytes())
    assert (q.height, q.width, q.bit_depth, q.range_size, q.domain_step, q.s_bits, q.o_bits) == \
        (H, W, bits, n, step, sb, ob)


def test_stream_header_rejects_foreign_or_inconsistent_headers():
    from oracle import oracle as O
    R = 256
    zero = dict(domain=np.zeros(R, np.int32), iso=np.zeros(R, np.uint8),
                s_idx=np.zeros(R, np.uint8), o_idx=np.zeros(R, np.uint8))
    good = O.stream_pack(64, 64, 4, 4, zero).tobytes()
    for at, val in [(0, ord("X")), (12, 9), (13, 3), (20, 7), (24, 5), (14, 0)]:
        bad = bytearray(good)
        bad[at] = val
        with pytest.raises(F.FicError) as e:
            F.stream_header(bytes(bad))
        assert e.value.status in (1, 2)
    with pytest.raises(F.FicError):
        F.stream_header(good[:16])


def test_stream_pack_and_unpack_validate_before_gpu_work():
    L = F.lib()
    p = F.Params(64, 64, 8, 4, 4).c()
    fake = ctypes.c_void_p(1 << 20)
    nb = F.stream_query(F.Params(64, 64, 8, 4, 4))[0]
    assert L.fic_stream_pack(ctypes.byref(p), None, fake, fake, fake, fake, nb, None) == 1
    assert L.fic_stream_pack(ctypes.byref(p), fake, fake, fake, fake, ctypes.c_void_p((1 << 20) + 2),
                             nb, None) == 1
    assert L.fic_stream_pack(ctypes.byref(p), fake, fake, fake, fake, fake, nb - 4, None) == 3
    assert L.fic_stream_unpack(ctypes.byref(p), fake, nb - 4, fake, fake, fake, fake, None) == 1
    assert L.fic_stream_unpack(ctypes.byref(p), None, nb, fake, fake, fake, fake, None) == 1


def test_quadtree_validates_before_gpu_work():
    L = F.lib()
    p = F.Params(256, 256, 8, 8, 4)
    nb, ml = F.quadtree_query(p, 4)
    assert ml == 4096 and nb > 0
    assert F.quadtree_query(p, 8)[1] == 1024
    for n_min, status in [(2, 2), (16, 1), (0, 2), (32, 2)]:
        with pytest.raises(F.FicError) as e:
            F.quadtree_query(p, n_min)
        assert e.value.status == status
    with pytest.raises(F.FicError) as e:
        F.quadtree_query(F.Params(256, 256, 8, 4, 4), 8)   # min above max
    assert e.value.status == 1
    fake = ctypes.c_void_p(1 << 20)
    codes = _lib._Codes(fake, fake, fake, fake, fake)
    out = _lib._QtOut(fake, fake, fake, codes, fake)
    cp = p.c()
    assert L.fic_encode_quadtree(ctypes.byref(cp), 4, ctypes.c_double(float("nan")), fake, out,
                                 fake, nb, None) == 1
    assert L.fic_encode_quadtree(ctypes.byref(cp), 4, ctypes.c_double(1.0), fake, out, fake,
                                 nb - 256, None) == 3
    assert L.fic_encode_quadtree(ctypes.byref(cp), 4, ctypes.c_double(1.0), None, out, fake,
                                 nb, None) == 1
