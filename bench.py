"""Benchmark of the PIFS range-domain search on one MI355X.

A step is one fic_encode of a 512x512 8-bit synthetic slice with 8x8 ranges
and 16x16 domains at stride 4, every range against every domain under the 8
transforms (4096 x 15,625 x 8 = 5.12e8 candidates, each through the FP16
contraction and the least-squares test): operand preparation, the search
with its fused fit/quantise/residual epilogue, and code extraction, with the
image already resident in HBM.  `value` is those candidates per second.

Secondary fields: the same slice with the shadow-block skip (flat ranges and
domains left out; its own evaluated count), the plain (direct) kernel on
identical work in both modes, the 512x512 12-bit slice at stride 2, the
paper's own workload shape (4x4 ranges) at its three image sizes beside its
Table III, the 256x256 decode workload (decoder, adjoint, refinement), the
64-slice batch, and the CPU oracle.  Prints one JSON line.
"""
import argparse
import csv
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_FP16_PEAK = 2.5e15  # dense FP16 MFMA FLOP/s of MI355X (AMD published)
MFMA_INT8_PEAK = 5.0e15  # dense int8 MFMA OP/s
HBM_PEAK = 8.0e12        # bytes/s
# hardware byte counters of the headline search kernel, from rocprofv3 --pmc
# (written by --pmc-summary); used only while the kernel sources are unchanged
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "search_u8_512_traffic.md")
SEARCH_SOURCES = ["fic_search_mfma.hip", "fic_search_common.h", "fic_device.h", "fic_internal.h"]
SEARCH_KERNEL = "k_search_mfma_u8<64>"


def search_source_hash():
    h = hashlib.sha256()
    for f in SEARCH_SOURCES:
        with open(os.path.join(ROOT, "paper_1404_0774_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic():
    """Scaled HBM bytes per launch of the search kernel, or None when no
    summary exists or the kernel changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    with open(TRAFFIC_PROFILE) as f:
        m = re.search(r"traffic: kernel=(\S+) fetch_bytes=(\d+) write_bytes=(\d+) src=(\w+)", f.read())
    if not m or m.group(4) != search_source_hash():
        return None
    return {"fetch": int(m.group(2)), "write": int(m.group(3))}


def pmc_summary(fetch_dir, write_dir):
    """Markdown summary of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of
    `bench.py --no-extras --copy-probe MIB`: KiB per dispatch, scaled by what
    the same counters read for the device-to-device copy of known size."""
    def per_kernel(d, counter):
        vals = {}
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"]
                vals.setdefault(name, []).append(float(r["Counter_Value"]))
        return vals
    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    copy_f = sum(sum(v) for k, v in fetch.items() if "copyBuffer" in k)
    copy_w = sum(sum(v) for k, v in write.items() if "copyBuffer" in k)
    copy_kib = 3 * 256 * 1024          # three copies of 256 MiB read and written
    sf = copy_kib / copy_f if copy_f else float("nan")
    sw = copy_kib / copy_w if copy_w else float("nan")
    lines = ["# HBM traffic per dispatch (rocprofv3 --pmc), 512x512 u8 encode", "",
             "Commands (from /tmp, TMPDIR=/tmp):", "",
             "    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <fetch_dir> -o run -- "
             "/usr/bin/python3 /root/repo/bench.py --steps 3 --warmup 1 --no-extras --no-cpu-baseline --copy-probe 256",
             "    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <write_dir> -o run -- (same program)",
             "    python bench.py --pmc-summary <fetch_dir> <write_dir>", "",
             f"Copy probe: 3 x 256 MiB device-to-device; FETCH_SIZE read {copy_f:.0f} KiB "
             f"(scale {sf:.3f}), WRITE_SIZE read {copy_w:.0f} KiB (scale {sw:.3f}).", "",
             "| kernel | dispatches | FETCH KiB | WRITE KiB | scaled read MB | scaled write MB |",
             "|---|---|---|---|---|---|"]
    search = None
    for name in sorted(set(fetch) | set(write)):
        if "fic::" not in name:
            continue
        f = sum(fetch.get(name, [0])) / max(1, len(fetch.get(name, [])))
        w = sum(write.get(name, [0])) / max(1, len(write.get(name, [])))
        short = name.split("(anonymous namespace)::", 1)[-1].split("(")[0]
        lines.append(f"| {short} | {len(fetch.get(name, []))} | {f:.1f} | {w:.1f} | "
                     f"{f * sf * 1024 / 1e6:.2f} | {w * sw * 1024 / 1e6:.2f} |")
        if short == SEARCH_KERNEL:
            search = (f * sf * 1024, w * sw * 1024)
    lines.append("")
    if search:
        lines.append(f"traffic: kernel={SEARCH_KERNEL} fetch_bytes={search[0]:.0f} "
                     f"write_bytes={search[1]:.0f} src={search_source_hash()}")
    return "\n".join(lines) + "\n"


def counters_summary(dirs):
    """Markdown summary of rocprofv3 --pmc runs of `bench.py --no-extras`
    (the full 512x512 u8 search): the SQ counters of the search kernel per
    wave, averaged over its dispatches."""
    vals = {}
    waves = None
    for d in dirs:
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if SEARCH_KERNEL not in r["Kernel_Name"].replace("(anonymous namespace)::", ""):
                    continue
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if "SQ_WAVES" in vals:
        waves = sum(vals["SQ_WAVES"]) / len(vals["SQ_WAVES"])
    lines = [f"# SQ counters of {SEARCH_KERNEL}, 512x512 u8 full search (rocprofv3 --pmc)", "",
             "Commands (from /tmp, TMPDIR=/tmp), one per counter group:", "",
             "    rocprofv3 --pmc <counters> --output-format csv -d <dir> -o run -- "
             "/usr/bin/python3 /root/repo/bench.py --steps 3 --warmup 1 --no-extras --no-cpu-baseline",
             "    python bench.py --counters-summary <dir> [<dir> ...]", "",
             f"Waves per dispatch: {waves:.0f}" if waves else "Waves per dispatch: (not collected)", "",
             "| counter | mean per dispatch | per wave |", "|---|---|---|"]
    for c in sorted(vals):
        m = sum(vals[c]) / len(vals[c])
        pw = f"{m / waves:.1f}" if waves else "-"
        lines.append(f"| {c} | {m:.0f} | {pw} |")
    lines += ["", "SQ_*_CYCLES, SQ_WAIT_* and SQ_ACTIVE_* count quad-cycles (4 clocks) summed "
              "over waves; SQ_VALU_MFMA_BUSY_CYCLES counts clocks summed over SIMDs (1024)."]
    return "\n".join(lines) + "\n"


def psnr(x, ref, peak):
    mse = float(((x - ref) ** 2).mean())
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)


def trace_summary(stats_dir, command):
    """Markdown table of a rocprofv3 --kernel-trace --stats run
    (run_kernel_stats.csv): calls and average duration per kernel."""
    rows = []
    with open(os.path.join(stats_dir, "run_kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["TotalDurationNs"]) / 1e3))
    rows.sort(key=lambda x: -x[3])
    lines = ["# Kernel durations (rocprofv3 --kernel-trace --stats)", "",
             "Command (from /tmp, TMPDIR=/tmp):", "", "    " + command, "",
             "| kernel | calls | average us | total us |", "|---|---|---|---|"]
    for name, calls, avg, tot in rows:
        short = name.split("(anonymous namespace)::", 1)[-1].split("(")[0]
        lines.append(f"| {short} | {calls} | {avg:.2f} | {tot:.1f} |")
    return "\n".join(lines) + "\n"


def time_encode(F, torch, timg, p, ws, steps, warmup):
    """Mean ms per fic_encode over `steps` back-to-back calls (two events
    around the whole run), then the per-phase split from a second run with
    the library's phase events (prep, seed, search, finalize) switched on."""
    dev = timg.device
    for _ in range(warmup):
        out = F.encode(timg, p, workspace=ws)
    torch.cuda.synchronize(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        out = F.encode(timg, p, workspace=ws)
    e1.record()
    torch.cuda.synchronize(dev)
    ms = e0.elapsed_time(e1) / steps
    F.timing_begin()
    for _ in range(steps):
        F.encode(timg, p, workspace=ws)
    torch.cuda.synchronize(dev)
    n, ms_prep, ms_seed, ms_search, ms_fin = F.timing_end()
    return out, ms, {"prep": ms_prep / n, "seed": ms_seed / n,
                     "search": ms_search / n, "finalize": ms_fin / n}


def codes_np(out):
    return {k: out[k].cpu().numpy() for k in ("domain", "iso", "s_idx", "o_idx", "err")}


# Table III of the paper: encode times of its own CUDA kernel and of a
# sequential CPU program, 4x4 ranges and 8x8 domains on a 4-pixel grid with
# the eight transforms, on its medical scans (not available here).  The units
# are not printed; seconds is the reading under which the GPU figures stay
# below that card's peak.
PAPER_TABLE3 = {
    "source": "Table III (encode time, CPU vs GPU; size reduction 40-41 %)",
    "gpu": "Fermi-class, compute capability 2.0, 16 SM x 32 = 512 cores at 1.30 GHz, 4 GB, CUDA 5.0",
    "cpu": "2.30 GHz, 64 KB L1D, 512 KB L2, 2 GB RAM, sequential program",
    "rows": [{"side": 256, "cpu_s": 247.432, "gpu_s": 0.232},
             {"side": 512, "cpu_s": 2369.4, "gpu_s": 3.521},
             {"side": 1024, "cpu_s": 39276.5, "gpu_s": 45.407}],
}


def mean_ms(torch, dev, fn, reps, warmup=2):
    """Mean milliseconds of fn() over `reps` back-to-back calls (events on
    the current stream around the whole run)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize(dev)
    return e0.elapsed_time(e1) / reps


def encode_line(F, torch, timg, p, ws, steps, warmup, k_flop):
    """One encode workload: codes, ms per call, phase split, the searched
    sub-table and the search kernel's achieved FLOP rate (k_flop FP16 MFMA
    FLOP per evaluated candidate; 0 for the plain method)."""
    out, ms, ph = time_encode(F, torch, timg, p, ws, steps, warmup)
    n_rs, n_ds = F.search_counts(out, p)
    ev = 8 * n_rs * n_ds
    line = {"ms_per_step": ms, "phases_ms": ph, "steps": steps,
            "ranges_searched": n_rs, "domains_searched": n_ds,
            "candidates_evaluated": ev, "evaluated_per_s": ev / (ms / 1e3)}
    if k_flop:
        line["search_tflops"] = k_flop * ev / (ph["search"] / 1e3) / 1e12
        line["search_mfma_frac"] = k_flop * ev / (ph["search"] / 1e3) / MFMA_FP16_PEAK
    return out, line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (full search, matrix cores)")
    ap.add_argument("--cpu-sample", type=int, default=4096, help="ranges timed on the CPU oracle")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the traffic summary of two rocprofv3 --pmc runs and exit")
    ap.add_argument("--counters-summary", nargs="+", metavar="PMC_DIR",
                    help="print the search kernel's SQ counters from rocprofv3 --pmc runs and exit")
    ap.add_argument("--trace-summary", nargs=2, metavar=("STATS_DIR", "COMMAND"),
                    help="print the kernel-duration summary of a rocprofv3 --stats run and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device-to-device three times (a kernel of "
                         "known traffic, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.pmc_summary:
        sys.stdout.write(pmc_summary(*args.pmc_summary))
        return
    if args.counters_summary:
        sys.stdout.write(counters_summary(args.counters_summary))
        return
    if args.trace_summary:
        sys.stdout.write(trace_summary(*args.trace_summary))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the search shards by ranges, see the design notes", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1404_0774_amd as F
    from fic_inputs import gen_image

    dev = torch.device("cuda:0")
    t_wall0 = time.time()

    # ---- headline: 512x512 u8, n = 8, stride 4, every candidate searched ------
    H = W = 512
    n, step, bits = 8, 4, 8
    img = gen_image(H, W, bits, 2)
    timg = torch.from_numpy(img).to(dev)
    p = F.Params(H, W, bits, n, step, method=F.METHOD_MFMA, full_search=1)
    R, ND, ws_bytes, _ = F.query(p)
    cand = 8 * R * ND
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    kf = 2.0 * n * n   # FP16 MFMA FLOP per candidate (one K-long inner product)

    out_m, full_m = encode_line(F, torch, timg, p, ws, args.steps, args.warmup, kf)
    assert full_m["candidates_evaluated"] == cand, "full search must visit every candidate"
    codes_m = codes_np(out_m)
    ms_m = full_m["ms_per_step"]
    flops = kf * cand
    achieved = flops / (full_m["phases_ms"]["search"] / 1e3)
    traffic = read_traffic()
    result = {
        "metric": "range-domain comparisons/s (MFMA GEMM vs direct) at bit-exact codes; decode PSNR",
        "value": cand / (ms_m / 1e3),
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
        "config": {"workload": "u8_512: 512x512 uint8 slice, 8x8 ranges, 16x16 domains stride 4, "
                               "every range against every domain (full search)",
                   "ranges": R, "domains": ND, "candidates": cand, "seed": 2},
        "phases_ms": full_m["phases_ms"],
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": MFMA_FP16_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / MFMA_FP16_PEAK,
                     "traffic": None if traffic is None else traffic["fetch"] + traffic["write"],
                     "kernel": SEARCH_KERNEL, "flop_per_launch": flops,
                     "candidates_per_launch": cand,
                     "note": "every (range, domain, transform) candidate goes through the FP16 "
                             "contraction and the least-squares test: 128 FLOP each"},
    }

    if not args.no_extras:
        # the same slice with the shadow-block skip: flat ranges and domains
        # have fixed outcomes and are left out of the contraction
        p.full_search = 0
        out_s, skip_m = encode_line(F, torch, timg, p, ws, args.steps, args.warmup, kf)
        same_skip = all(np.array_equal(codes_np(out_s)[k], codes_m[k]) for k in codes_m)
        # the plain method on identical work, in both modes
        p.method = F.METHOD_DIRECT
        dsteps = max(2, args.steps // 4)
        p.full_search = 1
        out_d, full_d = encode_line(F, torch, timg, p, ws, dsteps, 1, 0)
        p.full_search = 0
        out_ds, skip_d = encode_line(F, torch, timg, p, ws, dsteps, 1, 0)
        same_d = all(np.array_equal(codes_np(o)[k], codes_m[k]) for o in (out_d, out_ds)
                     for k in codes_m)
        result["skip_flat"] = dict(skip_m, note="ranges and domains without variance left out "
                                   "(their outcome is fixed); value = evaluated candidates / s",
                                   codes_identical_to_full=bool(same_skip))
        result["direct"] = {"full": full_d, "skip_flat": skip_d}
        result["mfma_over_direct"] = full_d["ms_per_step"] / ms_m
        result["mfma_over_direct_skip_flat"] = skip_d["ms_per_step"] / skip_m["ms_per_step"]
        result["mfma_over_direct_search_kernel"] = (full_d["phases_ms"]["search"]
                                                    / full_m["phases_ms"]["search"])
        result["codes_identical_mfma_direct"] = bool(same_d)
        p.method, p.full_search = F.METHOD_MFMA, 1

        s, o = F.dequantize(out_m["s_idx"], out_m["o_idx"], p)
        traj = F.decode(out_m["domain"], out_m["iso"], s.contiguous(), o.contiguous(), p, 12, 128.0)
        x = traj[-1].double().cpu().numpy()
        ref = img.astype(np.float64)
        result["decode_psnr_db"] = {"T": 12, "unclamped": psnr(x, ref, 255.0),
                                    "clamped_rounded": psnr(np.clip(np.rint(x), 0, 255), ref, 255.0)}

        # ---- 512x512 12-bit, n = 8, stride 2 ------------------------------------
        img12 = gen_image(512, 512, 12, 3)
        t12 = torch.from_numpy(img12.astype(np.int16)).to(dev)
        p12 = F.Params(512, 512, 12, 8, 2, method=F.METHOD_MFMA, full_search=1)
        R12, ND12, ws12b, _ = F.query(p12)
        ws12 = torch.empty(ws12b + 256, dtype=torch.uint8, device=dev)
        c12 = 8 * R12 * ND12
        kf12 = 4 * 2.0 * 64   # four FP16 partial products (hi/lo planes) per candidate
        st12 = max(3, args.steps // 4)
        o12, full12 = encode_line(F, torch, t12, p12, ws12, st12, 2, kf12)
        p12.full_search = 0
        o12s, skip12 = encode_line(F, torch, t12, p12, ws12, st12, 2, kf12)
        # the same contraction on the int8 matrix cores (4 int8 products of
        # K = 64 per candidate, against the 5.0 POP/s int8 peak)
        p12.method, p12.full_search = F.METHOD_MFMA_I8, 1
        ws12i = torch.empty(F.query(p12)[2] + 256, dtype=torch.uint8, device=dev)
        o12i, full12i = encode_line(F, torch, t12, p12, ws12i, st12, 2, 0)
        full12i["search_int8_tops"] = 4 * 2.0 * 64 * c12 / (full12i["phases_ms"]["search"] / 1e3) / 1e12
        full12i["search_int8_frac"] = full12i["search_int8_tops"] * 1e12 / MFMA_INT8_PEAK
        p12.full_search = 0
        o12is, skip12i = encode_line(F, torch, t12, p12, ws12i, st12, 2, 0)
        p12.method, p12.full_search = F.METHOD_DIRECT, 1
        o12d, full12d = encode_line(F, torch, t12, p12, ws12, 2, 1, 0)
        p12.full_search = 0
        o12ds, skip12d = encode_line(F, torch, t12, p12, ws12, 2, 1, 0)
        ref12 = codes_np(o12)
        same12 = all(np.array_equal(codes_np(o)[k], ref12[k])
                     for o in (o12s, o12d, o12ds, o12i, o12is) for k in ref12)
        result["ct12_512"] = {
            "workload": "512x512 12-bit slice, 8x8 ranges, 16x16 domains stride 2",
            "candidates": c12, "value": c12 / (full12["ms_per_step"] / 1e3),
            "unit": "comparisons/s", "full": full12, "skip_flat": skip12,
            "int8": {"full": full12i, "skip_flat": skip12i,
                     "over_fp16_full": full12["ms_per_step"] / full12i["ms_per_step"]},
            "direct": {"full": full12d, "skip_flat": skip12d},
            "mfma_over_direct": full12d["ms_per_step"] / full12["ms_per_step"],
            "mfma_over_direct_skip_flat": skip12d["ms_per_step"] / skip12["ms_per_step"],
            "codes_identical_all_modes_and_methods": bool(same12)}

        # ---- quadtree ranges: 8x8 split into 4x4 where the residual is high ----
        qt = []
        for tau in (10.0, 40.0):
            pq = F.Params(H, W, bits, 8, step, method=F.METHOD_MFMA, full_search=1)
            qout = F.encode_quadtree(timg, pq, 4, tau)
            nleaf = int(qout["y"].numel())
            n4 = int((qout["size"] == 4).sum())
            ms_q = mean_ms(torch, dev, lambda: F.encode_quadtree(timg, pq, 4, tau), 5, 1)
            # candidates evaluated: all 8x8 ranges, then the 4x4 quadrants of
            # the split ones, each against every domain of its side
            ev = 8 * R * ND + 8 * n4 * F.query(F.Params(H, W, bits, 4, step))[1]
            qt.append({"tau": tau, "leaves": nleaf, "leaves_4x4": n4, "ms": ms_q,
                       "candidates_evaluated": ev, "evaluated_per_s": ev / (ms_q / 1e3)})
        result["quadtree"] = {"workload": "512x512 uint8, 8x8 ranges split into 4x4 quadrants "
                                          "when the residual exceeds tau * n^2, domains on the "
                                          "4-pixel grid, full search per level",
                              "rows": qt}

        # ---- the paper's own workload shape: 4x4 ranges, 8x8 domains stride 4 ---
        pw = []
        for row in PAPER_TABLE3["rows"]:
            side = row["side"]
            pimg = torch.from_numpy(gen_image(side, side, 8, 7000 + side)).to(dev)
            pp = F.Params(side, side, 8, 4, 4, method=F.METHOD_MFMA, full_search=1)
            pR, pND, pwsb, _ = F.query(pp)
            pws = torch.empty(pwsb + 256, dtype=torch.uint8, device=dev)
            _, pl = encode_line(F, torch, pimg, pp, pws, max(3, args.steps // 4), 2, 2.0 * 16)
            pc = 8 * pR * pND
            pw.append({"side": side, "candidates": pc, "ms": pl["ms_per_step"],
                       "comparisons_per_s": pc / (pl["ms_per_step"] / 1e3),
                       "search_mfma_frac": pl["search_mfma_frac"],
                       "paper_gpu_s": row["gpu_s"], "paper_cpu_s": row["cpu_s"],
                       "paper_gpu_comparisons_per_s_if_seconds": pc / row["gpu_s"],
                       "speedup_over_paper_gpu_if_seconds": row["gpu_s"] / (pl["ms_per_step"] / 1e3)})
        result["paper_workloads"] = {
            "workload": "synthetic uint8 slices of the paper's sizes, 4x4 ranges, 8x8 domains "
                        "stride 4, full search (seed 7000 + side)",
            "rows": pw, "paper": PAPER_TABLE3}

        # ---- 256x256 u8, n = 4, stride 4: encode, decode, adjoint, refine ---------
        img5 = gen_image(256, 256, 8, 5)
        t5 = torch.from_numpy(img5).to(dev)
        p5 = F.Params(256, 256, 8, 4, 4, method=F.METHOD_MFMA, full_search=1)
        R5, ND5, ws5b, bw5 = F.query(p5)
        ws5 = torch.empty(ws5b + 256, dtype=torch.uint8, device=dev)
        o5, enc5 = encode_line(F, torch, t5, p5, ws5, args.steps, 2, 2.0 * 16)
        s5, o5v = F.dequantize(o5["s_idx"], o5["o_idx"], p5)
        s5, o5v = s5.contiguous(), o5v.contiguous()
        T = 12
        HW = 256 * 256
        tr5 = F.decode(o5["domain"], o5["iso"], s5, o5v, p5, T, 128.0)
        ms_dec = mean_ms(torch, dev, lambda: F.decode(o5["domain"], o5["iso"], s5, o5v, p5, T,
                                                      128.0), 20, 3)
        gxt = (2.0 * (tr5[-1] - t5.float()) / HW).contiguous()
        ms_bwd = mean_ms(torch, dev, lambda: F.decode_backward(o5["domain"], o5["iso"], s5, o5v,
                                                               tr5, gxt, p5), 20, 3)
        # algorithmic bytes: each iteration reads x_t and writes x_{t+1} once
        # (4 B each per pixel) and reads the codes (13 B per range); the
        # adjoint also reads the trajectory image and the domain->range table
        dec_bytes = T * (2 * 4 * HW + 13 * R5)
        bwd_bytes = T * (3 * 4 * HW + 13 * R5 + 4 * (ND5 + R5))
        scaled = {}
        for (num, den) in ((1, 2), (2, 1), (4, 1)):
            ms_z = mean_ms(torch, dev, lambda: F.decode_scaled(o5["domain"], o5["iso"], s5, o5v, p5,
                                                               (num, den), T, 128.0), 10, 2)
            hwz = HW * num * num // (den * den)
            zb = T * (2 * 4 * hwz + 13 * R5)
            scaled[f"{num}/{den}"] = {"side": 256 * num // den, "ms": ms_z,
                                      "gbps": zb / (ms_z / 1e3) / 1e9,
                                      "hbm_frac": zb / (ms_z / 1e3) / HBM_PEAK}
        # 64 different 256x256 slices (encoded by the batch encoder), decoded
        # together: one launch per iteration for all of them
        NB = 64
        dimgs = [torch.from_numpy(gen_image(256, 256, 8, 5000 + i)).to(dev) for i in range(NB)]
        dbat = F.Batch(dimgs, [F.Params(256, 256, 8, 4, 4) for _ in range(NB)])
        dcodes = dbat.run()
        torch.cuda.synchronize(dev)
        bd = torch.stack([c["domain"] for c in dcodes]).contiguous()
        bk = torch.stack([c["iso"] for c in dcodes]).contiguous()
        bsv, bov = F.dequantize(torch.stack([c["s_idx"] for c in dcodes]),
                                torch.stack([c["o_idx"] for c in dcodes]), p5)
        bsv, bov = bsv.contiguous(), bov.contiguous()
        ms_bdec = mean_ms(torch, dev, lambda: F.decode_batch(bd, bk, bsv, bov, p5, T, 128.0), 10, 2)
        bdec_bytes = NB * dec_bytes
        # the same 64 images' adjoint: one launch per reverse step for the batch
        btraj = F.decode_batch(bd, bk, bsv, bov, p5, T, 128.0)
        bgx = (torch.randn((NB, 256, 256), device=dev) * (2.0 / HW)).contiguous()
        ms_bbwd = mean_ms(torch, dev, lambda: F.decode_backward_batch(bd, bk, bsv, bov, btraj, bgx,
                                                                      p5), 10, 2)
        bbwd_bytes = NB * bwd_bytes
        del btraj, bgx
        del dbat, dimgs
        x0 = tr5[-1].double().cpu().numpy()
        ref5 = img5.astype(np.float64)
        sr, orf = s5.clone(), o5v.clone()
        t0 = time.time()
        loss = F.refine(o5["domain"], o5["iso"], sr, orf, t5, p5, iters=T, steps=50)
        torch.cuda.synchronize(dev)
        ms_ref = (time.time() - t0) * 1e3
        xr = F.decode(o5["domain"], o5["iso"], sr, orf, p5, T, 128.0)[-1].double().cpu().numpy()
        sq = torch.clamp(torch.floor((sr + 1.0) * 16 + 0.5), 0, 31)
        oq = torch.clamp(torch.floor((orf + 256.0) / 4 + 0.5), 0, 127)
        sqv, oqv = F.dequantize(sq.to(torch.uint8), oq.to(torch.uint8), p5)
        xq = F.decode(o5["domain"], o5["iso"], sqv.contiguous(), oqv.contiguous(), p5, T, 128.0)[-1].double().cpu().numpy()
        result["decode256"] = {
            "workload": "256x256 uint8, 4x4 ranges, 8x8 domains stride 4; decoder T = 12 from 128",
            "encode_value": 8 * R5 * ND5 / (enc5["ms_per_step"] / 1e3),
            "encode_ms": enc5["ms_per_step"],
            "decode_ms": ms_dec, "decode_gbps": dec_bytes / (ms_dec / 1e3) / 1e9,
            "decode_hbm_frac": dec_bytes / (ms_dec / 1e3) / HBM_PEAK,
            "adjoint_ms": ms_bwd, "adjoint_gbps": bwd_bytes / (ms_bwd / 1e3) / 1e9,
            "adjoint_hbm_frac": bwd_bytes / (ms_bwd / 1e3) / HBM_PEAK,
            "psnr_db": psnr(x0, ref5, 255.0),
            "scaled_decode": scaled,
            "batch_decode": {"images": NB, "ms": ms_bdec,
                             "gbps": bdec_bytes / (ms_bdec / 1e3) / 1e9,
                             "hbm_frac": bdec_bytes / (ms_bdec / 1e3) / HBM_PEAK,
                             "note": "64 different 256x256 slices with their own codes, "
                                     "one launch per iteration for the batch"},
            "batch_adjoint": {"images": NB, "ms": ms_bbwd,
                              "gbps": bbwd_bytes / (ms_bbwd / 1e3) / 1e9,
                              "hbm_frac": bbwd_bytes / (ms_bbwd / 1e3) / HBM_PEAK,
                              "note": "the same 64 slices' adjoint (tables built per call), "
                                      "one launch per reverse step for the batch"},
            "refine": {"steps": 50, "lr_s": 5e-3, "lr_o": 0.5, "ms": ms_ref,
                       "loss_first": float(loss[0]), "loss_last": float(loss[-1]),
                       "psnr_db": psnr(xr, ref5, 255.0), "psnr_requantised_db": psnr(xq, ref5, 255.0)}}

        # ---- code stream: bytes per encode and the size reduction ---------------
        def stream_line(out, prm, raw_bytes):
            data = F.stream_pack(out, prm)
            back = F.stream_unpack(data, prm)
            torch.cuda.synchronize(dev)
            ok = all(torch.equal(back[k], out[k]) for k in ("domain", "iso", "s_idx", "o_idx"))
            nb, B = F.stream_query(prm)
            return {"bytes": nb, "record_bits": B, "raw_bytes": raw_bytes,
                    "ratio": raw_bytes / nb, "size_reduction": 1.0 - nb / raw_bytes,
                    "pack_ms": mean_ms(torch, dev, lambda: F.stream_pack(out, prm), 20),
                    "unpack_ms": mean_ms(torch, dev, lambda: F.stream_unpack(data, prm), 20),
                    "round_trip_identical": bool(ok)}
        p.full_search = 1
        result["stream"] = {
            "format": "32-byte header + one record per range: domain index (ceil(log2 N_d) "
                      "bits), transform (3), s index (5), o index (7)",
            "u8_512": stream_line(out_m, p, H * W),
            "ct12_512": stream_line(o12, F.Params(512, 512, 12, 8, 2), 512 * 512 * 12 // 8),
            "u8_256_n4": stream_line(o5, p5, 256 * 256),
            "paper_size_reduction": "40 % (256^2 and 512^2), 41 % (1024^2); 85 % when "
                                    "decoding at 4x the size (Table III and its text)"}

        # ---- 64 uneven slices, 8x8 ranges, 16x16 domains stride 8 ---------------
        from fic_inputs import batch_sides
        sides = batch_sides(64)
        bimgs = [torch.from_numpy(gen_image(sd, sd, 8, 4000 + i)).to(dev) for i, sd in enumerate(sides)]
        bcand = sum(8 * F.query(F.Params(sd, sd, 8, 8, 8))[0] * F.query(F.Params(sd, sd, 8, 8, 8))[1]
                    for sd in sides)
        batch_lines = {}
        for full in (1, 0):
            bparams = [F.Params(sd, sd, 8, 8, 8, full_search=full) for sd in sides]
            bat = F.Batch(bimgs, bparams)
            for _ in range(2):
                bat.run()
            torch.cuda.synchronize(dev)
            graph = torch.cuda.CUDAGraph()
            gs = torch.cuda.Stream(device=dev)
            gs.wait_stream(torch.cuda.current_stream(dev))
            with torch.cuda.stream(gs):
                with torch.cuda.graph(graph, stream=gs):
                    bat.run()
            torch.cuda.current_stream(dev).wait_stream(gs)
            torch.cuda.synchronize(dev)
            nrep = max(3, args.steps // 2)
            lat = []
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            total = 0.0
            for _ in range(nrep):
                e0.record()
                graph.replay()
                e1.record()
                torch.cuda.synchronize(dev)
                total += e0.elapsed_time(e1)
                tk = bat.ticks.cpu().numpy().astype(np.int64)
                lat.append((tk[1:] - tk[0]) / 100.0)   # 100 MHz ticks -> us
            ms_b = total / nrep
            lat = np.concatenate(lat)
            batch_lines[full] = {"ms_per_batch": ms_b, "slices_per_s": 64 / (ms_b / 1e3),
                                 "latency_us_p50": float(np.percentile(lat, 50)),
                                 "latency_us_p99": float(np.percentile(lat, 99))}
            del graph, bat
        result["batch64"] = {
            "workload": "64 uint8 slices, sides from {256..512}^2, 8x8 ranges, 16x16 domains "
                        "stride 8; one graph replay; full search",
            "slices": 64, "candidates": bcand,
            "value": bcand / (batch_lines[1]["ms_per_batch"] / 1e3), "unit": "comparisons/s",
            **batch_lines[1],
            "skip_flat": batch_lines[0],
            "latency_note": "device clock when each slice's codes were written minus the "
                            "start of the search launch"}

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        rs = np.arange(0, R, max(1, R // args.cpu_sample))
        t0 = time.time()
        ora = O.encode_ranges(img, n, step, rs)
        dt = time.time() - t0
        match = all(np.array_equal(ora[k], codes_m[k][rs]) for k in ora)
        result["cpu_baseline"] = {"value": len(rs) * 8 * ND / dt, "unit": "comparisons/s",
                                  "cores": O.max_threads(), "kind": "oracle",
                                  "sample": f"{len(rs)} of {R} ranges of the same slice, full domain search each; {dt:.1f} s",
                                  "codes_match_gpu": bool(match)}
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize(dev)
        result["copy_probe_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
    result["wall_s"] = time.time() - t_wall0
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
