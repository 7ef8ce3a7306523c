"""The code stream on the GPU against the oracle's bit-by-bit writer and
reader: identical bytes, identical codes back, and the codes of real encodes
surviving the round trip (the decode of the unpacked codes is the decode of
the encoded ones)."""
import numpy as np
import pytest
import torch

import paper_1404_0774_amd as F
from oracle import oracle as O
from fic_inputs import gen_image

pytestmark = pytest.mark.gpu
FIELDS = ("domain", "iso", "s_idx", "o_idx")


def to_dev(codes):
    return {k: torch.from_numpy(np.ascontiguousarray(codes[k])).cuda() for k in FIELDS}


@pytest.mark.parametrize("H,W,bits,n,step,sb,ob,seed", [
    (64, 64, 8, 4, 4, 5, 7, 1),        # 27-bit records
    (512, 512, 8, 8, 4, 5, 7, 2),      # 15,625 domains: 29-bit records
    (512, 512, 12, 8, 2, 5, 7, 3),     # 62,001 domains: 31-bit records
    (40, 56, 8, 4, 3, 3, 6, 4),        # ragged
    (16, 16, 8, 8, 8, 1, 1, 5),        # one domain: D = 0, 5-bit records
    (256, 256, 8, 4, 4, 8, 8, 6),      # 31-bit records, full index fields
])
def test_pack_and_unpack_match_the_oracle(H, W, bits, n, step, sb, ob, seed):
    rng = np.random.default_rng(seed)
    R, nd = (H // n) * (W // n), O.n_domains(H, W, n, step)
    codes = dict(domain=rng.integers(0, nd, R).astype(np.int32), iso=rng.integers(0, 8, R).astype(np.uint8),
                 s_idx=rng.integers(0, 2 ** sb, R).astype(np.uint8),
                 o_idx=rng.integers(0, 2 ** ob, R).astype(np.uint8))
    codes["domain"][-1], codes["s_idx"][-1], codes["o_idx"][-1] = nd - 1, 2 ** sb - 1, 2 ** ob - 1
    p = F.Params(H, W, bits, n, step, s_bits=sb, o_bits=ob)
    ref = O.stream_pack(H, W, n, step, codes, bits=bits, s_bits=sb, o_bits=ob)
    got = F.stream_pack(to_dev(codes), p)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), ref)
    back = F.stream_unpack(torch.from_numpy(ref).cuda(), F.stream_header(ref.tobytes()))
    torch.cuda.synchronize()
    for k in FIELDS:
        np.testing.assert_array_equal(back[k].cpu().numpy(), codes[k])


def test_encoded_slice_round_trips_to_the_same_decode():
    H = W = 256
    img = torch.from_numpy(gen_image(H, W, 8, 5)).cuda()
    p = F.Params(H, W, 8, 4, 4)
    out = F.encode(img, p)
    data = F.stream_pack(out, p)
    back = F.stream_unpack(data)
    torch.cuda.synchronize()
    for k in FIELDS:
        assert torch.equal(back[k], out[k]), k
    s, o = F.dequantize(back["s_idx"], back["o_idx"], p)
    s0, o0 = F.dequantize(out["s_idx"], out["o_idx"], p)
    a = F.decode(back["domain"], back["iso"], s.contiguous(), o.contiguous(), p, 12, 128.0)
    b = F.decode(out["domain"], out["iso"], s0.contiguous(), o0.contiguous(), p, 12, 128.0)
    assert torch.equal(a, b)
    # 4096 ranges x (12 + 3 + 5 + 7) bits = 13,824 bytes + header, from 65,536
    assert data.numel() == 32 + 13824
