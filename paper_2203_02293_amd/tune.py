"""Autotuner of the solve kernel's tile (columns per workgroup).

For each representative shape (columns, layers, bins) and precision it times
rt_solve_fluxes with every admissible tile width K (K * bins <= 512) and
records the fastest in ``tuning.json`` next to this file.  The binding
(``rt.tuned_cols_per_block``) picks the entry nearest to a request's shape.

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

SHAPES = [  # (columns, layers, bins): GCM size, serving mix corners, high resolution
    (2562, 40, 30), (512, 40, 30), (4096, 120, 30), (256, 80, 100), (2048, 60, 100),
    (1024, 80, 300), (4096, 120, 300),
]


def candidates(nb: int, n_cols: int) -> list[int]:
    ks = [k for k in (1, 2, 3, 4, 6, 8, 12, 16, 24, 32) if k * nb <= 512 and k <= n_cols]
    return ks or [1]


def time_one(s, inp, out, precision, k, reps, torch):
    for _ in range(3):
        s.solve(inp, precision=precision, out=out, cols_per_block=k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        s.solve(inp, precision=precision, out=out, cols_per_block=k)
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
            times = {k: time_one(s, inp, out, prec, k, args.reps, torch) for k in candidates(NB, C)}
            best = min(times, key=times.get)
            entries.append(dict(n_cols=C, n_layers=N, n_bins=NB, precision=prec,
                                cols_per_block=best, ms=times[best]))
            report.append(dict(shape=[C, N, NB], precision=prec,
                               ms={str(k): round(v, 4) for k, v in times.items()}, best=best))
            print(f"[tune] {C}x{N}x{NB} prec={prec}: " +
                  " ".join(f"K={k}:{v:.3f}ms" for k, v in times.items()) + f" -> {best}",
                  file=sys.stderr, flush=True)
        s.close()
        del inp, out
        torch.cuda.empty_cache()
    doc = dict(created=time.strftime("%Y-%m-%d %H:%M:%S"), entries=entries, sweeps=report)
    pathlib.Path(args.out).write_text(json.dumps(doc, indent=1))
    print(json.dumps(doc))


if __name__ == "__main__":
    main()
