"""Pins for the oracle's code stream (the codes saved to the encoding file,
Section IV; the size reduction of Table III).  The paper defines no file
format, so the stream's bytes are pinned against a record worked out by hand
from the format's definition, its size against the closed form, and its
reading against its writing."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from fic_inputs import gen_image


@pytest.mark.parametrize("nd,bits", [(1, 0), (2, 1), (3, 2), (4, 2), (5, 3), (8, 3), (9, 4),
                                     (3969, 12), (15625, 14), (62001, 16), (65536, 16),
                                     (65537, 17)])
def test_domain_index_bits(nd, bits):
    assert O.stream_domain_bits(nd) == bits


@pytest.mark.parametrize("H,W,n,step,sb,ob", [(64, 64, 4, 4, 5, 7), (512, 512, 8, 4, 5, 7),
                                              (512, 512, 8, 2, 5, 7), (40, 56, 4, 3, 3, 6),
                                              (16, 16, 8, 8, 1, 1), (256, 256, 4, 4, 8, 8)])
def test_size_closed_form(H, W, n, step, sb, ob):
    R = (H // n) * (W // n)
    nd = ((H - 2 * n) // step + 1) * ((W - 2 * n) // step + 1)
    B = math.ceil(math.log2(nd)) + 3 + sb + ob if nd > 1 else 3 + sb + ob
    assert O.stream_bytes(H, W, n, step, sb, ob) == 32 + 4 * math.ceil(R * B / 32)


def test_hand_worked_records():
    # 16x16, 4x4 ranges, 8x8 domains at stride 4: 16 ranges, 9 domains, so a
    # record is 4 + 3 + 5 + 7 = 19 bits.  Range 0: domain 5, transform 3,
    # contrast 16, offset 64; range 1: domain 8, transform 7, contrast 31,
    # offset 127; the rest zero.  Bits from stream bit 0 (field LSB first):
    #   r0: 1010 110 00001 0000001        r1 (from bit 19): 0001 111 11111 1111111
    # bytes (bit 0 = LSB): 00110101=0x35  00001000=0x08  (bits 16..23)
    # 0,0,1 | 0,0,0,1,1 -> 0b11000100=0xC4; bits 24..31: 1,1,1,1,1,1,1,1 -> 0xFF;
    # bits 32..37: 1,1,1,1,1,1 then 0,0 -> 0x3F; everything after is zero
    H = W = 16
    codes = dict(domain=np.zeros(16, np.int32), iso=np.zeros(16, np.uint8),
                 s_idx=np.zeros(16, np.uint8), o_idx=np.zeros(16, np.uint8))
    codes["domain"][:2] = [5, 8]
    codes["iso"][:2] = [3, 7]
    codes["s_idx"][:2] = [16, 31]
    codes["o_idx"][:2] = [64, 127]
    data = O.stream_pack(H, W, 4, 4, codes)
    header = (b"PIFS" + (16).to_bytes(4, "little") + (16).to_bytes(4, "little") + bytes([8, 4, 5, 7])
              + (4).to_bytes(4, "little") + bytes([4, 0, 0, 0]) + (16).to_bytes(8, "little"))
    assert bytes(data[:32]) == header
    payload = np.zeros(40, np.uint8)        # 16 x 19 = 304 bits -> 10 words
    payload[:5] = [0x35, 0x08, 0xC4, 0xFF, 0x3F]
    np.testing.assert_array_equal(data[32:], payload)


@pytest.mark.parametrize("H,W,n,step,sb,ob", [(64, 64, 4, 4, 5, 7), (40, 56, 4, 3, 3, 6),
                                              (48, 64, 8, 2, 8, 8), (16, 16, 8, 8, 1, 1)])
def test_round_trip_random_and_extreme_codes(H, W, n, step, sb, ob):
    rng = np.random.default_rng(H + W + sb)
    R = (H // n) * (W // n)
    nd = O.n_domains(H, W, n, step)
    codes = dict(domain=rng.integers(0, nd, R).astype(np.int32), iso=rng.integers(0, 8, R).astype(np.uint8),
                 s_idx=rng.integers(0, 2 ** sb, R).astype(np.uint8),
                 o_idx=rng.integers(0, 2 ** ob, R).astype(np.uint8))
    codes["domain"][0], codes["iso"][0], codes["s_idx"][0], codes["o_idx"][0] = nd - 1, 7, 2 ** sb - 1, 2 ** ob - 1
    data = O.stream_pack(H, W, n, step, codes, s_bits=sb, o_bits=ob)
    back = O.stream_unpack(H, W, n, step, data, s_bits=sb, o_bits=ob)
    for k in codes:
        np.testing.assert_array_equal(back[k], codes[k])


def test_pack_rejects_codes_outside_their_fields():
    H = W = 32; n = 4; step = 4
    R, nd = 64, O.n_domains(H, W, n, step)
    ok = dict(domain=np.zeros(R, np.int32), iso=np.zeros(R, np.uint8),
              s_idx=np.zeros(R, np.uint8), o_idx=np.zeros(R, np.uint8))
    for field, bad in [("domain", nd), ("iso", 8), ("s_idx", 32), ("o_idx", 128)]:
        c = {k: v.copy() for k, v in ok.items()}
        c[field][3] = bad
        with pytest.raises(ValueError):
            O.stream_pack(H, W, n, step, c)


def test_encoded_codes_survive_the_stream():
    H = W = 64; n = 4; step = 4
    img = gen_image(H, W, 8, 31)
    c = O.encode(img, n, step)
    data = O.stream_pack(H, W, n, step, c)
    back = O.stream_unpack(H, W, n, step, data)
    for k in back:
        np.testing.assert_array_equal(back[k], c[k])
    # 256 ranges x (8 + 3 + 5 + 7) bits = 5,888 bits -> 736 bytes + header
    assert len(data) == 32 + 736
