"""Autotuner of the solve launch: kernel (lane, layer or deep) and tile width.

For each representative shape (columns, layers, bins) and precision it times
rt_solve_fluxes with each kernel and every admissible tile width K and
records the fastest in ``tuning.json`` next to this file.  The binding
(``rt.tuned_launch``) picks the entry nearest to a request's shape.

    python -m paper_2203_02293_amd.tune [--quick]
"""
from __future__ import annotations

import argparse
import json
import pathlib
import sys
import time

import numpy as np

from . import rt, synth

SHAPES = [  # (columns, layers, bins): GCM size, serving mix corners, high resolution,
    # few deep columns
    (2562, 40, 30), (512, 40, 30), (4096, 120, 30), (256, 80, 100), (2048, 60, 100),
    (1024, 80, 300), (4096, 120, 300), (10242, 80, 300), (1, 4096, 30), (16, 1000, 30),
    (64, 400, 30),
]


def candidates(nb: int, n_cols: int) -> list[tuple[int, int]]:
    """(kernel, K) pairs: the layer kernel's default tile and a spread around it,
    the lane kernel's tiles (K * bins <= 512) and the deep kernel."""
    out = [(rt.RT_KERNEL_LAYER, 0), (rt.RT_KERNEL_DEEP, 0)]
    out += [(rt.RT_KERNEL_LAYER, k) for k in (1, 2, 3, 4, 6, 8, 10, 11, 12, 16, 24, 32)
            if k * nb <= 1024 and k <= n_cols]
    out += [(rt.RT_KERNEL_LANE, k) for k in (1, 2, 4, 8, 16)
            if k * nb <= 512 and k <= n_cols]
    return out


def time_one(s, inp, out, precision, cand, reps, torch):
    kernel, k = cand
    try:
        s.solve(inp, precision=precision, out=out, cols_per_block=k, kernel=kernel)
    except rt.RtError:
        return None    # tile does not fit this kernel (LDS)
    for _ in range(2):
        s.solve(inp, precision=precision, out=out, cols_per_block=k, kernel=kernel)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        s.solve(inp, precision=precision, out=out, cols_per_block=k, kernel=kernel)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="only the GCM-size shape")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--out", default=str(rt.TUNING_PATH))
    args = ap.parse_args(argv)
    import torch
    shapes = SHAPES[:1] if args.quick else SHAPES
    entries, report = [], []
    for (C, N, NB) in shapes:
        spec = synth.Spec(name="tune", g_level=5, n_layers=N, n_bins=NB, cloud="night", seed=77)
        w = synth.make(spec, n_cols=C)
        s = rt.Solver(w["lambda_edges"], w["F_star"])
        inp = rt.to_device(w)
        out = s.outputs(C, N)
        for prec in (rt.RT_FP64, rt.RT_MIXED):
            times = {}
            for cand in candidates(NB, C):
                t = time_one(s, inp, out, prec, cand, args.reps, torch)
                if t is not None:
                    times[cand] = t
            best = min(times, key=times.get)
            entries.append(dict(n_cols=C, n_layers=N, n_bins=NB, precision=prec,
                                kernel=best[0], cols_per_block=best[1], ms=times[best]))
            name = {rt.RT_KERNEL_LANE: "lane", rt.RT_KERNEL_LAYER: "layer",
                    rt.RT_KERNEL_DEEP: "deep"}
            report.append(dict(shape=[C, N, NB], precision=prec,
                               ms={f"{name[kk]}:{k}": round(v, 4) for (kk, k), v in times.items()},
                               best=[name[best[0]], best[1]]))
            print(f"[tune] {C}x{N}x{NB} prec={prec}: " +
                  " ".join(f"{name[kk]}:K={k}:{v:.3f}ms" for (kk, k), v in times.items()) +
                  f" -> {name[best[0]]}:{best[1]}", file=sys.stderr, flush=True)
        s.close()
        del inp, out
        torch.cuda.empty_cache()
    doc = dict(created=time.strftime("%Y-%m-%d %H:%M:%S"), entries=entries, sweeps=report)
    pathlib.Path(args.out).write_text(json.dumps(doc, indent=1))
    print(json.dumps(doc))


if __name__ == "__main__":
    main()
