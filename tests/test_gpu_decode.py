"""GPU decoder and adjoint against the FP64 oracle, finite differences and
bitwise reproducibility."""
import numpy as np
import pytest
import torch

import paper_1404_0774_amd as F
from oracle import oracle as O
from fic_inputs import gen_image

pytestmark = pytest.mark.gpu


def codes_for(H, W, n, step, seed):
    img = gen_image(H, W, 8, seed)
    c = O.encode(img, n, step)
    s, o = O.dequantize(c["s_idx"], c["o_idx"])
    return img, c["domain"], c["iso"], s, o


def dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)


@pytest.mark.parametrize("H,W,n,step", [(64, 64, 4, 4), (96, 64, 8, 2), (40, 56, 4, 3)])
def test_decode_matches_oracle(H, W, n, step):
    img, d, k, s, o = codes_for(H, W, n, step, 31)
    p = F.Params(H, W, 8, n, step)
    T = 12
    traj = F.decode(dev(d, torch.int32), dev(k, torch.uint8), dev(s, torch.float32),
                    dev(o, torch.float32), p, T, 128.0).cpu().numpy()
    ref = O.decode(H, W, n, step, d, k, s, o, T, 128.0)
    # FP32 iteration of a map with |s| <= 1: error grows at most ~T ulps of 2^8
    assert np.abs(traj - ref).max() <= 1e-3


def test_decode_and_adjoint_256_workload_match_oracle():
    """The 256x256 workload (4x4 ranges, 8x8 domains at stride 4, T = 12 from
    128): the oracle's codes decoded on the GPU against the FP64 decoder,
    every pixel of every iterate, and the adjoint against the FP64 gradient
    and central differences of the FP64 decoder."""
    H = W = 256
    n, step, T = 4, 4, 12
    img, d, k, s, o = codes_for(H, W, n, step, 5)
    p = F.Params(H, W, 8, n, step)
    dd, kd = dev(d, torch.int32), dev(k, torch.uint8)
    sd, od = dev(s, torch.float32), dev(o, torch.float32)
    traj = F.decode(dd, kd, sd, od, p, T, 128.0)
    ref = O.decode(H, W, n, step, d, k, s, o, T, 128.0)
    assert np.abs(traj.cpu().numpy() - ref).max() <= 1e-3
    target = img.astype(np.float64)
    g = 2.0 * (traj[-1] - torch.from_numpy(target).float().cuda()) / (H * W)
    gs, go = F.decode_backward(dd, kd, sd, od, traj, g, p)
    gs, go = gs.cpu().numpy().astype(np.float64), go.cpu().numpy().astype(np.float64)
    rg = 2.0 * (ref[-1] - target) / (H * W)
    rs, ro = O.decode_backward(H, W, n, step, d, k, s, o, T, ref, rg)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(gs, rs) <= 1e-4 and rel(go, ro) <= 1e-4
    rng = np.random.default_rng(6)
    idx = rng.choice(len(s), 64, replace=False)
    loss = lambda ss, oo: (((O.decode(H, W, n, step, d, k, ss, oo, T, 128.0)[-1] - target) ** 2).mean())
    fs, fo = [], []
    for r in idx:
        sp, sm = s.copy(), s.copy(); sp[r] += 1e-4; sm[r] -= 1e-4
        fs.append((loss(sp, o) - loss(sm, o)) / 2e-4)
        op, om = o.copy(), o.copy(); op[r] += 1e-2; om[r] -= 1e-2
        fo.append((loss(s, op) - loss(s, om)) / 2e-2)
    assert rel(gs[idx], np.array(fs)) <= 1e-3 and rel(go[idx], np.array(fo)) <= 1e-3


@pytest.mark.parametrize("num,den", [(1, 2), (2, 1), (4, 1), (1, 1)])
def test_decode_scaled_matches_oracle(num, den):
    """The 256x256 workload's codes (4x4 ranges, 8x8 domains at stride 4)
    decoded at 1/2, 2 and 4 times the size, every pixel of every iterate
    against the FP64 oracle; the 1x case equals fic_decode bit for bit."""
    H = W = 256
    n, step, T = 4, 4, 12
    img, d, k, s, o = codes_for(H, W, n, step, 5)
    p = F.Params(H, W, 8, n, step)
    dd, kd = dev(d, torch.int32), dev(k, torch.uint8)
    sd, od = dev(s, torch.float32), dev(o, torch.float32)
    traj = F.decode_scaled(dd, kd, sd, od, p, (num, den), T, 128.0).cpu().numpy()
    ref = O.decode_scaled(H, W, n, step, num, den, d, k, s, o, T, 128.0)
    assert traj.shape == ref.shape == (T + 1, H * num // den, W * num // den)
    assert np.abs(traj - ref).max() <= 1e-3
    if num == den:
        base = F.decode(dd, kd, sd, od, p, T, 128.0).cpu().numpy()
        assert np.array_equal(traj, base)


@pytest.mark.parametrize("T", [1, 2, 5])
@pytest.mark.parametrize("H,W,n,step", [(64, 64, 4, 4), (96, 64, 8, 4), (96, 64, 8, 2),
                                        (40, 56, 4, 3), (36, 44, 4, 2)])
def test_range_pooled_decode_equals_per_pixel_decode(H, W, n, step, T):
    """fic_decode pools each range's domain cells once (16-byte accesses when
    rows, domain corners and range rows sit on 4-float boundaries, single
    floats otherwise); every iterate equals the generic per-pixel decode
    (fic_decode_scaled at 1/1) bit for bit."""
    img, d, k, s, o = codes_for(H, W, n, step, 33)
    p = F.Params(H, W, 8, n, step)
    args = (dev(d, torch.int32), dev(k, torch.uint8), dev(s, torch.float32),
            dev(o, torch.float32))
    a = F.decode(*args, p, T, 128.0)
    b = F.decode_scaled(*args, p, (1, 1), T, 128.0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("B", [3, 8])
@pytest.mark.parametrize("H,W,n,step", [(64, 64, 4, 4), (96, 64, 8, 2)])
def test_decode_batch_matches_single_decodes_and_oracle(H, W, n, step, B):
    """B images of one geometry with their own codes in one batched decode
    (B = 8 takes the XCD-grouped workgroup order): each trajectory equals
    fic_decode's bit for bit and the FP64 oracle's within 1e-3."""
    T = 12
    cs = [codes_for(H, W, n, step, 50 + b) for b in range(B)]
    p = F.Params(H, W, 8, n, step)
    stack = lambda i, dt: dev(np.stack([c[i] for c in cs]), dt)
    traj = F.decode_batch(stack(1, torch.int32), stack(2, torch.uint8), stack(3, torch.float32),
                          stack(4, torch.float32), p, T, 128.0)
    torch.cuda.synchronize()
    assert traj.shape == (B, T + 1, H, W)
    for b, (img, d, k, s, o) in enumerate(cs):
        one = F.decode(dev(d, torch.int32), dev(k, torch.uint8), dev(s, torch.float32),
                       dev(o, torch.float32), p, T, 128.0)
        assert torch.equal(traj[b], one), b
        ref = O.decode(H, W, n, step, d, k, s, o, T, 128.0)
        assert np.abs(traj[b].cpu().numpy() - ref).max() <= 1e-3


def test_decode_16x16_ranges_matches_oracle():
    H, W, n, step, T = 128, 96, 16, 8, 12
    img = gen_image(H, W, 8, 52)
    c = O.encode(img, n, step)
    s, o = O.dequantize(c["s_idx"], c["o_idx"])
    p = F.Params(H, W, 8, n, step)
    traj = F.decode(dev(c["domain"], torch.int32), dev(c["iso"], torch.uint8),
                    dev(s, torch.float32), dev(o, torch.float32), p, T, 128.0).cpu().numpy()
    ref = O.decode(H, W, n, step, c["domain"], c["iso"], s, o, T, 128.0)
    assert np.abs(traj - ref).max() <= 1e-3


def test_decode_scaled_rejects_fractional_pixels():
    p = F.Params(64, 64, 8, 4, 4)
    z = torch.zeros(256, dtype=torch.int32, device="cuda")
    u = torch.zeros(256, dtype=torch.uint8, device="cuda")
    f = torch.zeros(256, dtype=torch.float32, device="cuda")
    for scale in [(1, 8), (1, 3), (3, 8), (0, 1)]:
        with pytest.raises((F.FicError, ValueError)):
            F.decode_scaled(z, u, f, f, p, scale, 2, 128.0)


def test_backward_matches_fp64_gradient_and_fd():
    H = W = 64
    n, step, T = 4, 4, 12
    img, d, k, s, o = codes_for(H, W, n, step, 32)
    s = np.clip(s, -0.9375, 0.9375)
    p = F.Params(H, W, 8, n, step)
    target = img.astype(np.float64)
    sd, od = dev(s, torch.float32), dev(o, torch.float32)
    traj = F.decode(dev(d, torch.int32), dev(k, torch.uint8), sd, od, p, T, 128.0)
    g = 2.0 * (traj[-1] - torch.from_numpy(target).float().cuda()) / (H * W)
    gs, go = F.decode_backward(dev(d, torch.int32), dev(k, torch.uint8), sd, od, traj, g, p)
    gs, go = gs.cpu().numpy().astype(np.float64), go.cpu().numpy().astype(np.float64)
    # FP64 reference gradient of the same loss
    rtraj = O.decode(H, W, n, step, d, k, s, o, T, 128.0)
    rg = 2.0 * (rtraj[-1] - target) / (H * W)
    rs, ro = O.decode_backward(H, W, n, step, d, k, s, o, T, rtraj, rg)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(gs, rs) <= 1e-4 and rel(go, ro) <= 1e-4
    # central differences of the FP64 decoder on 64 seeded coordinates each
    rng = np.random.default_rng(3)
    idx = rng.choice(len(s), 64, replace=False)
    loss = lambda ss, oo: (((O.decode(H, W, n, step, d, k, ss, oo, T, 128.0)[-1] - target) ** 2).mean())
    fs, fo = [], []
    for r in idx:
        sp, sm = s.copy(), s.copy(); sp[r] += 1e-4; sm[r] -= 1e-4
        fs.append((loss(sp, o) - loss(sm, o)) / 2e-4)
        op, om = o.copy(), o.copy(); op[r] += 1e-2; om[r] -= 1e-2
        fo.append((loss(s, op) - loss(s, om)) / 2e-2)
    assert rel(gs[idx], np.array(fs)) <= 1e-3 and rel(go[idx], np.array(fo)) <= 1e-3


@pytest.mark.parametrize("case", ["one_domain", "few_domains", "ragged_rect",
                                  "odd_step", "n8_step4", "n8_step8",
                                  "many_ranges", "single_domain_image",
                                  "one_domain_column"])
def test_backward_shared_domains(case):
    """Many ranges on one domain (heavy units, each summed by a workgroup),
    the in-LDS sort (up to 8,192 ranges and 16,384 domains) and the radix
    sort beyond it, 2x2-cell units (even STEP) and pixel units (odd STEP),
    with at most 2 x 2 covering domains (STEP >= n) or more."""
    rng = np.random.default_rng(41)
    H, W, n, step = {"one_domain": (64, 48, 4, 4),      # 165 domains
                     "few_domains": (128, 96, 4, 2),    # 2,745 domains
                     "ragged_rect": (264, 272, 4, 1),   # 68,105 domains: radix sort
                     "odd_step": (72, 64, 4, 5),        # pixel units, 2 x 2 cover
                     "n8_step4": (128, 128, 8, 4),      # 8x8 ranges, 4 x 4 cover
                     "n8_step8": (128, 96, 8, 8),       # 8x8 ranges, 2 x 2 cover
                     "many_ranges": (512, 512, 4, 8),   # 16,384 ranges: radix sort
                     "single_domain_image": (8, 8, 4, 4),  # one domain, no sort pass
                     "one_domain_column": (16, 8, 4, 3),   # 1 x 3 domains, pixel units
                     }[case]
    p = F.Params(H, W, 8, n, step)
    R, ND = F.query(p)[:2]
    if case == "one_domain":
        d = np.zeros(R, dtype=np.int32)
    elif case == "few_domains":
        d = rng.choice(np.array([0, 5, ND - 1], dtype=np.int32), R)
    else:
        d = rng.integers(0, ND, R).astype(np.int32)
        d[: R // 3] = min(7, ND - 1)              # one long list among many short
    k = rng.integers(0, 8, R).astype(np.uint8)
    s = rng.uniform(-0.8, 0.8, R)
    o = rng.uniform(-40, 200, R)
    T = 6
    target = rng.integers(0, 256, (H, W)).astype(np.float64)
    sd, od = dev(s, torch.float32), dev(o, torch.float32)
    traj = F.decode(dev(d, torch.int32), dev(k, torch.uint8), sd, od, p, T, 128.0)
    g = 2.0 * (traj[-1] - torch.from_numpy(target).float().cuda()) / (H * W)
    gs, go = F.decode_backward(dev(d, torch.int32), dev(k, torch.uint8), sd, od, traj, g, p)
    gs2, go2 = F.decode_backward(dev(d, torch.int32), dev(k, torch.uint8), sd, od, traj, g, p)
    assert torch.equal(gs, gs2) and torch.equal(go, go2)
    s32 = s.astype(np.float32).astype(np.float64)
    o32 = o.astype(np.float32).astype(np.float64)
    rtraj = O.decode(H, W, n, step, d, k, s32, o32, T, 128.0)
    rg = 2.0 * (rtraj[-1] - target) / (H * W)
    rs, ro = O.decode_backward(H, W, n, step, d, k, s32, o32, T, rtraj, rg)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(gs.cpu().numpy().astype(np.float64), rs) <= 1e-4
    assert rel(go.cpu().numpy().astype(np.float64), ro) <= 1e-4


@pytest.mark.parametrize("H,W,n,step", [(64, 48, 4, 4), (96, 64, 8, 2), (40, 56, 4, 3)])
def test_backward_batch_matches_single_calls(H, W, n, step):
    """The batched adjoint: every image's dL/ds, dL/do bitwise equal to the
    single call's, with one image of the batch on a single shared domain
    (heavy units) and the others random."""
    rng = np.random.default_rng(77)
    p = F.Params(H, W, 8, n, step)
    R, ND = F.query(p)[:2]
    B, T = 5, 6
    d = rng.integers(0, ND, (B, R)).astype(np.int32)
    d[2] = 0
    k = rng.integers(0, 8, (B, R)).astype(np.uint8)
    s = rng.uniform(-0.8, 0.8, (B, R)).astype(np.float32)
    o = rng.uniform(-40, 200, (B, R)).astype(np.float32)
    dd, kd, sd, od = dev(d, torch.int32), dev(k, torch.uint8), dev(s, torch.float32), dev(o, torch.float32)
    traj = F.decode_batch(dd, kd, sd, od, p, T, 128.0)
    g = dev(rng.normal(size=(B, H, W)), torch.float32)
    gs, go = F.decode_backward_batch(dd, kd, sd, od, traj, g, p)
    for b in range(B):
        s1, o1 = F.decode_backward(dd[b], kd[b], sd[b], od[b], traj[b].contiguous(), g[b], p)
        assert torch.equal(gs[b], s1) and torch.equal(go[b], o1), b
    # and one image against the FP64 gradient
    rtraj = O.decode(H, W, n, step, d[1], k[1], s[1].astype(np.float64), o[1].astype(np.float64),
                     T, 128.0)
    rs, ro = O.decode_backward(H, W, n, step, d[1], k[1], s[1].astype(np.float64),
                               o[1].astype(np.float64), T, rtraj,
                               g[1].cpu().numpy().astype(np.float64))
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(gs[1].cpu().numpy().astype(np.float64), rs) <= 1e-4
    assert rel(go[1].cpu().numpy().astype(np.float64), ro) <= 1e-4


def test_backward_bitwise_reproducible_and_autograd():
    H = W = 64
    n, step, T = 4, 2, 12
    img, d, k, s, o = codes_for(H, W, n, step, 33)
    p = F.Params(H, W, 8, n, step)
    dd, kk = dev(d, torch.int32), dev(k, torch.uint8)
    sd = dev(s, torch.float32).requires_grad_(True)
    od = dev(o, torch.float32).requires_grad_(True)
    tgt = torch.from_numpy(img.astype(np.float32)).cuda()
    outs = []
    for _ in range(3):
        sd.grad = None; od.grad = None
        x = F.FicDecode.apply(sd, od, dd, kk, p, T, 128.0)
        loss = ((x - tgt) ** 2).mean()
        loss.backward()
        outs.append((sd.grad.clone(), od.grad.clone()))
    for a in outs[1:]:
        assert torch.equal(a[0], outs[0][0]) and torch.equal(a[1], outs[0][1])


def test_zero_iterations():
    H = W = 32
    img, d, k, s, o = codes_for(H, W, 4, 4, 34)
    p = F.Params(H, W, 8, 4, 4)
    sd, od = dev(s, torch.float32), dev(o, torch.float32)
    traj = F.decode(dev(d, torch.int32), dev(k, torch.uint8), sd, od, p, 0, 77.0)
    assert traj.shape[0] == 1 and bool((traj == 77.0).all())
    gs, go = F.decode_backward(dev(d, torch.int32), dev(k, torch.uint8), sd, od, traj,
                               torch.ones_like(traj[0]), p)
    assert bool((gs == 0).all()) and bool((go == 0).all())


def _adam_reference(s, o, gs, go, lr_s, lr_o, t=1, b1=0.9, b2=0.999, eps=1e-8):
    m_s, v_s = (1 - b1) * gs, (1 - b2) * gs * gs
    m_o, v_o = (1 - b1) * go, (1 - b2) * go * go
    c1, c2 = 1 - b1 ** t, 1 - b2 ** t
    s1 = np.clip(s - lr_s * (m_s / c1) / (np.sqrt(v_s / c2) + eps), -0.999, 0.999)
    o1 = o - lr_o * (m_o / c1) / (np.sqrt(v_o / c2) + eps)
    return s1, o1


def test_refine_one_step_is_adam_on_adjoint_gradient():
    H = W = 64
    n, step, T = 4, 4, 12
    img, d, k, s, o = codes_for(H, W, n, step, 35)
    p = F.Params(H, W, 8, n, step)
    dd, kk = dev(d, torch.int32), dev(k, torch.uint8)
    s0, o0 = dev(s, torch.float32), dev(o, torch.float32)
    timg = torch.from_numpy(img).cuda()
    traj = F.decode(dd, kk, s0, o0, p, T, 128.0)
    g = 2.0 * (traj[-1] - timg.float()) / (H * W)
    gs, go = F.decode_backward(dd, kk, s0, o0, traj, g, p)
    s1, o1 = s0.clone(), o0.clone()
    loss = F.refine(dd, kk, s1, o1, timg, p, iters=T, steps=1, lr_s=5e-3, lr_o=0.5)
    rs, ro = _adam_reference(s0.cpu().numpy().astype(np.float64), o0.cpu().numpy().astype(np.float64),
                             gs.cpu().numpy().astype(np.float64), go.cpu().numpy().astype(np.float64),
                             5e-3, 0.5)
    np.testing.assert_allclose(s1.cpu().numpy(), rs, rtol=0, atol=1e-5)
    np.testing.assert_allclose(o1.cpu().numpy(), ro, rtol=0, atol=1e-4)
    mse0 = float(((traj[-1].double() - timg.double()) ** 2).mean())
    assert abs(float(loss[0]) - mse0) <= 1e-9 * max(1.0, mse0)


def test_refine_lowers_attractor_error_and_is_reproducible():
    H = W = 64
    n, step, T = 4, 4, 12
    img, d, k, s, o = codes_for(H, W, n, step, 36)
    p = F.Params(H, W, 8, n, step)
    dd, kk = dev(d, torch.int32), dev(k, torch.uint8)
    timg = torch.from_numpy(img).cuda()
    runs = []
    for _ in range(2):
        s1, o1 = dev(s, torch.float32), dev(o, torch.float32)
        loss = F.refine(dd, kk, s1, o1, timg, p, iters=T, steps=50)
        runs.append((s1.cpu(), o1.cpu(), loss.cpu()))
    loss = runs[0][2].numpy()
    assert loss[-1] < loss[0]
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    assert torch.equal(runs[0][2], runs[1][2])
    assert bool((runs[0][0].abs() <= 0.999).all())
