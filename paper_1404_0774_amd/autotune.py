"""Launch-shape autotuner for libfic.

Times fic_encode (and the batched encode) over a small grid of launch shapes
on the current GPU and writes the fastest ones as a JSON table that the
library reads at load (``tuning.json`` beside libfic.so, or
``fic_load_tuning``).  Every shape yields the same codes; the tuner checks
that too, so a shape that changed a code would stop it.

    python -m paper_1404_0774_amd.autotune [--out PATH] [--reps N]

Workloads: the 512x512 8-bit slice with 8x8 ranges at domain stride 4 (both
methods), the 512x512 12-bit slice at stride 2 (FP16 and int8 matrix-core
searches), the 256x256 8-bit slice with 4x4 ranges, and a batch of 64 uneven
8-bit slices at stride 8.
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import _lib as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _images():
    sys.path.insert(0, ROOT)
    from fic_inputs import batch_sides, gen_image
    return gen_image, batch_sides


def _time(fn, reps, dev):
    """Median milliseconds of fn() over reps runs (each bracketed by events)."""
    fn()
    torch.cuda.synchronize(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize(dev)
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def _codes(out):
    return [out[k].cpu().numpy() for k in ("domain", "iso", "s_idx", "o_idx", "err")]


def tune_single(name, img, p, chunk_grid, seed_grid, reps, dev, log):
    """Sweep (col_chunks, seed_blocks) for one encode; returns the best entry."""
    R, ND, wsb, _ = F.query(p)
    ws = torch.empty(wsb + 256, dtype=torch.uint8, device=dev)
    F.set_tuning([])
    ref = _codes(F.encode(img, p, workspace=ws))
    base = F.get_tuning(p)
    sweep = []
    best = None
    for seed in seed_grid:
        for ch in chunk_grid:
            entry = dict(bit_depth=p.bit_depth, range_size=p.range_size, method=p.method,
                         min_domains=0, col_chunks=ch, seed_blocks=seed)
            F.set_tuning([entry])
            got = F.get_tuning(p)
            if (got["col_chunks"], got["seed_blocks"]) != (ch, seed):
                continue  # clamped to a shape already covered
            ms = _time(lambda: F.encode(img, p, workspace=ws), reps, dev)
            codes = _codes(F.encode(img, p, workspace=ws))
            if not all(np.array_equal(a, b) for a, b in zip(codes, ref)):
                raise RuntimeError(f"{name}: shape chunks={ch} seed={seed} changed the codes")
            sweep.append({"col_chunks": ch, "seed_blocks": seed, "ms": ms})
            if best is None or ms < best[0]:
                best = (ms, ch, seed)
    F.set_tuning([])
    ms_default = _time(lambda: F.encode(img, p, workspace=ws), reps, dev)
    log(f"{name}: default chunks={base['col_chunks']} seed={base['seed_blocks']} "
        f"{ms_default:.4f} ms; best chunks={best[1]} seed={best[2]} {best[0]:.4f} ms")
    entry = dict(bit_depth=p.bit_depth, range_size=p.range_size, method=p.method,
                 min_domains=ND, col_chunks=best[1], seed_blocks=best[2], item_blocks=0)
    record = {"workload": name, "ms_default": ms_default, "ms_best": best[0],
              "sweep": sweep}
    return entry, record


def tune_batch(imgs, params, item_grid, seed_grid, reps, dev, log):
    """Sweep (item_blocks, seed_blocks) for the batched encode."""
    F.set_tuning([])
    ref = [_codes(c) for c in F.Batch(imgs, params).run()]
    sweep = []
    best = None
    for seed in seed_grid:
        for ib in item_grid:
            F.set_tuning([dict(bit_depth=8, range_size=params[0].range_size, method=F.METHOD_MFMA,
                               min_domains=0, seed_blocks=seed, item_blocks=ib)])
            bat = F.Batch(imgs, params)
            ms = _time(bat.run, reps, dev)
            for c, r in zip(bat.run(), ref):
                if not all(np.array_equal(a, b) for a, b in zip(_codes(c), r)):
                    raise RuntimeError(f"batch: item_blocks={ib} seed={seed} changed the codes")
            sweep.append({"item_blocks": ib, "seed_blocks": seed, "ms": ms})
            if best is None or ms < best[0]:
                best = (ms, ib, seed)
    F.set_tuning([])
    bat = F.Batch(imgs, params)
    ms_default = _time(bat.run, reps, dev)
    log(f"batch64: default {ms_default:.4f} ms; best item_blocks={best[1]} seed={best[2]} "
        f"{best[0]:.4f} ms")
    entry = dict(bit_depth=8, range_size=params[0].range_size, method=F.METHOD_MFMA,
                 min_domains=0, col_chunks=0, seed_blocks=best[2], item_blocks=best[1])
    return entry, {"workload": "batch64", "ms_default": ms_default, "ms_best": best[0],
                   "sweep": sweep}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=F.TUNING_PATH)
    ap.add_argument("--reps", type=int, default=15)
    ap.add_argument("--skip-direct", action="store_true")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    gen_image, batch_sides = _images()
    t0 = time.time()

    def log(msg):
        print(f"[autotune {time.time() - t0:6.1f}s] {msg}", flush=True)

    F.lib()
    entries, records = [], []
    chunks = [2, 3, 4, 6, 8, 12, 16, 24, 32]
    img = torch.from_numpy(gen_image(512, 512, 8, 2)).to(dev)
    e, r = tune_single("u8_512 mfma", img, F.Params(512, 512, 8, 8, 4), chunks, [0, 1, 2, 4, 8],
                       args.reps, dev, log)
    entries.append(e); records.append(r)
    if not args.skip_direct:
        # the plain method is tuned on the full search, the work it is
        # compared on with the matrix-core search
        e, r = tune_single("u8_512 direct", img,
                           F.Params(512, 512, 8, 8, 4, method=F.METHOD_DIRECT, full_search=1),
                           [4, 6, 8, 12, 16, 32], [1], max(3, args.reps // 3), dev, log)
        entries.append(e); records.append(r)
    img12 = torch.from_numpy(gen_image(512, 512, 12, 3).astype(np.int16)).to(dev)
    e, r = tune_single("ct12_512 mfma", img12, F.Params(512, 512, 12, 8, 2), [2, 4, 8, 12, 16, 20, 24, 32],
                       [1, 2, 4, 8], max(3, args.reps // 3), dev, log)
    entries.append(e); records.append(r)
    e, r = tune_single("ct12_512 mfma_i8", img12,
                       F.Params(512, 512, 12, 8, 2, method=F.METHOD_MFMA_I8),
                       [2, 4, 8, 12, 16, 20, 24, 32], [1, 2, 4, 8], max(3, args.reps // 3), dev, log)
    entries.append(e); records.append(r)
    img5 = torch.from_numpy(gen_image(256, 256, 8, 5)).to(dev)
    e, r = tune_single("u8_256 n4 mfma", img5, F.Params(256, 256, 8, 4, 4), chunks, [0, 1, 2, 4],
                       args.reps, dev, log)
    entries.append(e); records.append(r)
    sides = batch_sides(64)
    bimgs = [torch.from_numpy(gen_image(s, s, 8, 4000 + i)).to(dev) for i, s in enumerate(sides)]
    bparams = [F.Params(s, s, 8, 8, 8) for s in sides]
    batch_entry, r = tune_batch(bimgs, bparams, [8, 16, 32, 64, 128, 256], [0, 1, 2, 4],
                                max(3, args.reps // 3), dev, log)
    entries.append(batch_entry); records.append(r)

    # the batch entry applies from 0 domains; single-slice entries carry the
    # batch's item length so that the batch keeps it for large slices too
    for en in entries:
        if en["bit_depth"] == 8 and en["range_size"] == 8 and en["method"] == F.METHOD_MFMA:
            en["item_blocks"] = batch_entry["item_blocks"]
    doc = {"device": torch.cuda.get_device_name(dev), "reps": args.reps,
           "entries": entries, "records": records}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    F.load_tuning(args.out)
    log(f"wrote {len(entries)} entries to {args.out}")


if __name__ == "__main__":
    main()
