"""Benchmark of the range-domain search on one MI355X.

A step is one fic_encode of a 512x512 8-bit synthetic slice with 8x8 ranges
and 16x16 domains at stride 4 (4096 ranges x 15,625 domains x 8 transforms =
5.12e8 candidate comparisons): operand preparation, the matrix-core search
with its fused fit/quantise/residual epilogue, and code extraction, with the
image already resident in HBM.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_FP16_PEAK = 2.5e15  # dense FP16 MFMA FLOP/s of MI355X (AMD published)
HBM_PEAK = 8.0e12        # bytes/s


def psnr(x, ref, peak):
    mse = float(((x - ref) ** 2).mean())
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=512, help="ranges timed on the CPU oracle")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the search shards by ranges, see the design notes", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1404_0774_amd as F
    from fic_inputs import gen_image

    dev = torch.device("cuda:0")
    H = W = 512
    n, step, bits = 8, 4, 8
    img = gen_image(H, W, bits, 2)
    timg = torch.from_numpy(img).to(dev)
    p = F.Params(H, W, bits, n, step, method=F.METHOD_MFMA)
    R, ND, ws_bytes, _ = F.query(p)
    cand = 8 * R * ND
    K = n * n
    flops = 2.0 * K * cand            # MFMA FLOPs of the search contraction
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)

    def run(method, steps):
        p.method = method
        for _ in range(args.warmup):
            out = F.encode(timg, p, workspace=ws)
        torch.cuda.synchronize(dev)
        F.timing_begin()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            out = F.encode(timg, p, workspace=ws)
        e1.record()
        torch.cuda.synchronize(dev)
        ncalls, ms_prep, ms_search, ms_fin = F.timing_end()
        total = e0.elapsed_time(e1)
        return out, total / steps, ms_prep / ncalls, ms_search / ncalls, ms_fin / ncalls

    t_wall0 = time.time()
    out_m, ms_m, prep_m, search_m, fin_m = run(F.METHOD_MFMA, args.steps)
    codes_m = {k: out_m[k].cpu().numpy() for k in ("domain", "iso", "s_idx", "o_idx", "err")}
    dsteps = max(2, args.steps // 4)
    out_d, ms_d, prep_d, search_d, fin_d = run(F.METHOD_DIRECT, dsteps)
    codes_d = {k: out_d[k].cpu().numpy() for k in ("domain", "iso", "s_idx", "o_idx", "err")}
    same = all(np.array_equal(codes_m[k], codes_d[k]) for k in codes_m)

    # decode quality of the codes (12 iterations from mid-grey, FP32)
    p.method = F.METHOD_MFMA
    s, o = F.dequantize(out_m["s_idx"], out_m["o_idx"], p)
    traj = F.decode(out_m["domain"], out_m["iso"], s.contiguous(), o.contiguous(), p, 12, 128.0)
    x = traj[-1].double().cpu().numpy()
    ref = img.astype(np.float64)
    ps_raw = psnr(x, ref, 255.0)
    ps_q = psnr(np.clip(np.rint(x), 0, 255), ref, 255.0)

    value = cand / (ms_m / 1e3)
    achieved = flops / (search_m / 1e3)
    result = {
        "metric": "range-domain comparisons/s (MFMA GEMM vs direct) at bit-exact codes; decode PSNR",
        "value": value,
        "unit": "comparisons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_m,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16",
        "data": "synthetic",
        "config": {"workload": "u8_512: 512x512 uint8 slice, 8x8 ranges, 16x16 domains stride 4",
                   "ranges": R, "domains": ND, "candidates": cand, "seed": 2},
        "phases_ms": {"prep": prep_m, "search": search_m, "finalize": fin_m},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": MFMA_FP16_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / MFMA_FP16_PEAK, "traffic": None,
                     "kernel": "search (matrix-core contraction + fused epilogue)",
                     "flop_per_launch": flops},
        "direct": {"value": cand / (ms_d / 1e3), "ms_per_step": ms_d, "search_ms": search_d,
                   "steps": dsteps},
        "mfma_over_direct": ms_d / ms_m,
        "codes_identical_mfma_direct": bool(same),
        "decode_psnr_db": {"T": 12, "unclamped": ps_raw, "clamped_rounded": ps_q},
    }

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        rs = np.arange(0, R, max(1, R // args.cpu_sample))
        t0 = time.time()
        ora = O.encode_ranges(img, n, step, rs)
        dt = time.time() - t0
        match = all(np.array_equal(ora[k], codes_m[k][rs]) for k in ora)
        result["cpu_baseline"] = {"value": len(rs) * 8 * ND / dt, "unit": "comparisons/s",
                                  "cores": O.max_threads(), "kind": "oracle",
                                  "sample": f"{len(rs)} of {R} ranges (every {R // len(rs)}th), full domain search each; {dt:.1f} s",
                                  "codes_match_gpu": bool(match)}
    result["wall_s"] = time.time() - t_wall0
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
