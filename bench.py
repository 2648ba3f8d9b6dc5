"""Benchmark of the improved two-stream solve on one MI355X.

One step = one rt_solve_fluxes over the whole GCM-size workload (2562
icosahedral columns x 40 layers x 30 bins: Planck sources, coefficients,
beam, Thomas solve, bin sums, net flux and heating) with every input already
resident in HBM.  Default: FP64; the mixed-precision path is timed the same
way and reported beside it.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-mixed]
                  [--no-serving] [--no-cfg4]

Prints ONE JSON line.  Besides the headline FP64 figure and the mixed path
beside it, the default run adds the serving mix (saturation, then p50/p99 at
50 % and 80 % of it) and the 10242 x 80 x 300 high-resolution solve.  Only
the ``cpu_baseline`` leg runs the CPU oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import pathlib
import sys
import time

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TF = 78.6            # MI355X FP64 vector
FP32_PEAK_TF = 157.3           # MI355X FP32 vector
# VALU issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles
# (16 lanes wide), at 2.4 GHz
VALU_ISSUE_PEAK_G = 256 * 4 / 4 * 2.4
WORKLOADS = {
    "cfg1": "GCM size: 2562 icosahedral columns x 40 layers x 30 bins log-spaced 0.3-30 um, "
            "night-side cloud deck",
    "cfg4": "high resolution: 10242 icosahedral columns x 80 layers x 300 bins log-spaced "
            "0.3-30 um, cloud decks to w0 0.9999 / g0 0.98, dtau log-uniform [1e-8, 1e3]",
    "cfg1_kdist": "GCM size with k-distribution bins: 2562 icosahedral columns x 40 layers x "
                  "30 bins x 20 Gaussian points (600 solves per column), night-side cloud deck",
    "cfg1_sub": "GCM size on the sub-layer grid: 2562 icosahedral columns x 40 layers split "
                "at their centres (80 slabs) x 30 bins, night-side cloud deck",
    "cfg1_optics": "the paper's radiative step at GCM size: 2562 columns x 40 layers on the "
                   "sub-layer grid (80 slabs) x 30 bins x 20 Gaussian points; optical "
                   "properties from a synthetic 60 T x 28 p k-table with Rayleigh and "
                   "condensates, then the solve",
    "deep1": "one deep column: 1 dayside column (mu_star 0.85) x 4096 layers x 30 bins, "
             "cloud deck",
    "deep16": "few deep columns: 16 columns x 1000 layers x 30 bins, day and night, about "
              "half with cloud decks",
}
METRIC = "two-stream column·bin solves/s (FP64 vs mixed, ≤1e-5 rel err); p50/p99 latency"


def algorithmic_bytes(C: int, N: int, NB: int) -> int:
    """Bytes one solve must move at least: every input read once, every
    (bin-summed) output written once."""
    inputs = 3 * 8 * N * C * NB + 2 * 8 * (N + 1) * C + 2 * 8 * C
    outputs = 4 * 8 * (N + 1) * C + 2 * 8 * N * C + 8 * C * NB + 4 * C
    return inputs + outputs


def kernel_source_hash() -> str:
    """Hash of the sources the lane and layer kernels are compiled from."""
    h = hashlib.sha256()
    csrc = ROOT / "paper_2203_02293_amd" / "csrc"
    for name in ("rt_internal.hpp", "rt_kernels.hip", "rt_math.hpp", "rt_physics.hpp", "rt_wave.hpp"):
        h.update((csrc / name).read_bytes())
    return h.hexdigest()[:16]


def _profiled(kernel: str, workload: str = "cfg1") -> dict | None:
    """The committed PMC summary of a kernel on a workload (2562x40x30 by
    default), if it was taken on the current kernel sources."""
    f = ROOT / "profiles" / f"traffic_{workload}.json"
    if not f.exists():
        return None
    d = json.loads(f.read_text())
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("kernels", {}).get(kernel)


def traffic_from_profiles(kernel: str, workload: str = "cfg1") -> float | None:
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size)."""
    k = _profiled(kernel, workload)
    return None if k is None else float(k["bytes_per_launch"])


def valu_issue(kernel: str, ms: float) -> dict | None:
    """VALU wave-instructions per launch (SQ_INSTS_VALU) over the launch time,
    against the issue peak: the limit this kernel actually runs into."""
    k = _profiled(kernel)
    if k is None or "valu_insts_per_launch" not in k:
        return None
    rate = k["valu_insts_per_launch"] / (ms * 1e-3) / 1e9
    return {"valu_insts": k["valu_insts_per_launch"], "achieved": rate, "peak": VALU_ISSUE_PEAK_G,
            "unit": "G wave-instructions/s", "frac": rate / VALU_ISSUE_PEAK_G}


def fp_rates(kernel: str, ms: float) -> dict | None:
    """Floating-point rate of a launch from the committed FLOP-mix counters
    (SQ_INSTS_VALU_{ADD,MUL,FMA}_F{32,64}, wave-instructions of 64 lanes, an FMA
    two flops) over the launch time, against the vector peaks (FP64 78.6, FP32
    157.3 TFLOP/s)."""
    k = _profiled(kernel)
    if k is None or "flops" not in k:
        return None
    f = k["flops"]
    out = {}
    for prec, peak in (("F64", FP64_PEAK_TF), ("F32", FP32_PEAK_TF)):
        fl = 64 * (f[f"SQ_INSTS_VALU_ADD_{prec}"] + f[f"SQ_INSTS_VALU_MUL_{prec}"]
                   + 2 * f[f"SQ_INSTS_VALU_FMA_{prec}"])
        tf = fl / (ms * 1e-3) / 1e12
        out[prec.lower()] = {"flops": fl, "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak}
    return out


def copy_bandwidth(torch, nbytes: int = 1 << 30, runs: int = 10) -> float:
    """Device-to-device copy rate (bytes read + bytes written per second, GB/s):
    the HBM rate a plain streaming kernel reaches on this device."""
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(runs):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / runs
    del src, dst
    return 2 * n * 8 / (ms * 1e-3) / 1e9


KERNEL_IDS = {"auto": None, "lane": 1, "layer": 2, "deep": 3}
KERNEL_NAMES = {1: "k_solve_lane", 2: "k_solve_layer", 3: "k_deep_*"}


def time_path(s, inp, out, precision, steps, warmup, torch, kernel=None, pre=None):
    """Warm up, then time exactly `steps` back-to-back steps on the current
    stream; a step is `pre()` (if given: the optical-properties step) and one
    solve."""
    stream = torch.cuda.current_stream()
    kw = {} if kernel is None else {"kernel": kernel, "cols_per_block": 0}
    for _ in range(warmup):
        if pre:
            pre()
        s.solve(inp, precision=precision, out=out, **kw)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        if pre:
            pre()
        s.solve(inp, precision=precision, out=out, **kw)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]   # ms, one launch each
    total_ms = ev[0].elapsed_time(ev[steps])
    return wall, total_ms, per


def pct(v, q):
    v = sorted(v)
    i = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[i]


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1


def time_oracle(work: dict, threads: int, runs: int) -> tuple[list, dict]:
    """Wall times of `runs` whole solves of `work` by the oracle on `threads`
    OpenMP threads (after one warm-up on a few columns), and the last result."""
    import oracle
    run = oracle.solve_sublayer if work.get("sublayer") else oracle.solve
    run(work, n_threads=threads, cols=(0, 16))
    times, ref = [], None
    for _ in range(runs):
        t0 = time.perf_counter()
        ref = run(work, n_threads=threads)
        times.append(time.perf_counter() - t0)
    return times, ref


def cpu_baseline(work, small: dict | None = None, runs: int = 5,
                 cfg4_sample: dict | None = None) -> tuple[dict, dict]:
    """The CPU oracle as it stands, timed on this host's cores: the median of
    `runs` whole FP64 solves of the benchmark workload on one thread and on all
    host threads, and the same for the small workload `small` if given.  The
    mixed-precision path has the same inputs and the same FP64 reference, so
    its CPU baseline is this one.  With `cfg4_sample` (1 % of the columns of the
    10242 x 80 x 300 workload) the same timings of the sample, and the whole
    workload's time extrapolated linearly in columns (stated as such).  Returns
    the timing block (headline value: all threads on the benchmark workload) and
    the oracle's outputs of the last all-thread solve."""
    threads = host_threads()
    nbg = lambda w: w["n_bins"] * w.get("n_gauss", 1)
    shape = lambda w: f"{w['n_cols']}x{w['n_layers']}x{nbg(w)}"
    per = {}
    ref = None
    for tag, w in (("small", small), ("workload", work), ("cfg4_sample", cfg4_sample)):
        if w is None:
            continue
        entry = {"shape": shape(w)}
        for nt in sorted({1, threads}):
            ts, r = time_oracle(w, nt, runs)
            med = float(np.median(ts))
            entry[f"{nt}_threads"] = {"median_s": med, "runs_s": ts,
                                      "value": w["n_cols"] * nbg(w) / med}
            if tag == "workload" and nt == threads:
                ref = r
        if tag == "cfg4_sample":
            entry["extrapolated"] = {f"{k}_s": v["median_s"] * 10242 / w["n_cols"]
                                     for k, v in entry.items() if k.endswith("_threads")}
            entry["note"] = ("1 % column sample (every 100th column) of 10242 x 80 x 300; "
                             "whole-workload times extrapolated linearly in columns")
        per[tag] = entry
        print(f"[bench] cpu baseline {entry['shape']}: " + ", ".join(
            f"{k} {v['median_s']:.3f} s" for k, v in entry.items() if k.endswith("_threads")),
            file=sys.stderr, flush=True)
    head = per["workload"][f"{threads}_threads"]
    return ({"value": head["value"], "unit": "column·bin solves/s", "cores": threads,
             "kind": "oracle", "cpu_model": cpu_model(),
             "sample": f"median of {runs} whole FP64 solves of the {per['workload']['shape']} "
                       f"workload on {threads} OpenMP threads (the mixed path shares its "
                       f"inputs and reference); single-thread and small-workload runs under "
                       f"'runs'",
             "runs": per}, ref)


def column_subset(work: dict, cols: np.ndarray) -> dict:
    """The workload restricted to some columns (columns are independent)."""
    w = dict(work, n_cols=int(cols.size))
    for k in ("p_iface", "T_iface"):
        w[k] = np.ascontiguousarray(work[k][:, cols])
    for k in ("dtau", "w0", "g0"):
        w[k] = np.ascontiguousarray(work[k][:, cols, :])
    for k in ("mu_star", "T_int"):
        w[k] = np.ascontiguousarray(work[k][cols])
    return w


def error_stats(got: dict, ref: dict, p_iface: np.ndarray, gravity: float = 47.0,
                floor: float = 1e-3) -> dict:
    """Errors of the bin-summed outputs against the oracle's, scaled as the parity
    tests scale them: S = the column's largest gross flux F_up + F_dn + F_beam;
    F_up, F_dn, F_beam by max(|ref|, floor S); F_net by S; heating Q by its flux
    divergence Q dp / g over S.  Max, p99 and median over (interface or layer,
    column)."""
    S = (ref["F_up"] + ref["F_dn"] + ref["F_beam"]).max(axis=0)
    e = {}
    for k in ("F_up", "F_dn", "F_beam"):
        e[k] = np.abs(got[k] - ref[k]) / np.maximum(np.abs(ref[k]), floor * S)
    e["F_net"] = np.abs(got["F_net"] - ref["F_net"]) / S
    dp = (p_iface[:-1] - p_iface[1:])
    e["heating"] = np.abs(got["heating"] - ref["heating"]) * dp / gravity / S
    return {k: {"max": float(v.max()), "p99": float(np.percentile(v, 99)),
                "median": float(np.median(v))} for k, v in e.items()}


def serving(args, torch, rt, synth) -> dict:
    """Serving mix: uneven requests (columns U{1..4096}, layers U{20..120}, bins in
    {30, 100, 300}, cloud fraction U[0, 0.5]) through rt_submit/rt_poll, half
    FP64 and half mixed, inputs resident on the device, one handle per spectral
    set-up; once with batched launches, once with the persistent worker.  For
    each: the saturation rate (every request submitted at time 0), then Poisson
    arrivals at the stated fractions of the batched saturation rate (the same
    arrival rates for both).  Latency = completion time (seen by polling) minus
    arrival time.  Every output slot's last result of a run is compared with the
    same request submitted alone on the same handle (bitwise)."""
    shapes = synth.serving_requests(args.serve_pool, seed=1003, max_cols=4096)
    pool = []
    for k, sh in enumerate(shapes):
        w = synth.make_request(sh)
        pool.append(dict(nb=w["n_bins"], lam=w["lambda_edges"], fs=w["F_star"], inp=rt.to_device(w),
                         C=w["n_cols"], N=w["n_layers"],
                         prec=rt.RT_FP64 if k % 2 == 0 else rt.RT_MIXED))
        del w
    torch.cuda.synchronize()

    def design(mode, rates, n_requests):
        solvers = {}
        for q in pool:
            if q["nb"] not in solvers:
                solvers[q["nb"]] = rt.Solver(q["lam"], q["fs"], max_inflight=256,
                                             hbm_budget_bytes=args.serve_budget_gib << 30,
                                             serve_mode=mode)
        # each request once alone (the reference of the bitwise check)
        for q in pool:
            s = solvers[q["nb"]]
            q["out"] = [s.outputs(q["C"], q["N"]) for _ in range(args.serve_copies)]
            torch.cuda.synchronize()
            if s.wait(s.submit(q["inp"], q["out"][0], q["prec"])) != rt.RT_OK:
                raise RuntimeError("serving request failed alone")
            q["alone"] = {k: q["out"][0][k].cpu().numpy() for k in ("F_net", "heating")}
            q["used"] = [False] * args.serve_copies

        def run(rate):
            """One run of n_requests requests; rate None: all arrive at once."""
            n = n_requests
            arrivals = (np.zeros(n) if rate is None
                        else synth.poisson_arrivals(n, rate, seed=int(rate)))
            order = np.random.Generator(np.random.PCG64(7 if rate is None else int(rate) + 1)
                                        ).integers(0, len(pool), n)
            busy = [[False] * args.serve_copies for _ in pool]
            inflight, lat, cb = {}, [], 0
            t0 = time.perf_counter()
            i = 0
            while i < n or inflight:
                now = time.perf_counter() - t0
                while i < n and arrivals[i] <= now:
                    q = pool[order[i]]
                    slot = next((m for m in range(args.serve_copies) if not busy[order[i]][m]), None)
                    if slot is None:      # every output copy of this request is busy: wait
                        break
                    busy[order[i]][slot] = True
                    t = solvers[q["nb"]].submit(q["inp"], q["out"][slot], q["prec"])
                    inflight[(q["nb"], t)] = (arrivals[i], order[i], slot)
                    i += 1
                for key in list(inflight):
                    nb, t = key
                    st = solvers[nb].poll(t)
                    if st == rt.RT_PENDING:
                        continue
                    if st != rt.RT_OK:
                        raise RuntimeError(f"serving request failed: status {st}")
                    arr, qi, slot = inflight.pop(key)
                    lat.append(time.perf_counter() - t0 - arr)
                    busy[qi][slot] = False
                    pool[qi]["used"][slot] = True
                    cb += pool[qi]["C"] * pool[qi]["nb"]
            el = time.perf_counter() - t0
            torch.cuda.synchronize()
            checked = equal = 0
            for q in pool:
                for m, used in enumerate(q["used"]):
                    if used:
                        checked += 1
                        equal += all(np.array_equal(q["out"][m][k].cpu().numpy(), q["alone"][k])
                                     for k in ("F_net", "heating"))
                    q["used"][m] = False
            return {"rate_hz": None if rate is None else rate, "requests": len(lat),
                    "requests_per_s": len(lat) / el, "p50_ms": pct(lat, 50) * 1e3,
                    "p99_ms": pct(lat, 99) * 1e3, "solves_per_s": cb / el, "seconds": el,
                    "results_checked": checked, "results_equal_alone": equal}

        name = "persistent" if mode == rt.RT_SERVE_PERSISTENT else "batched"
        sat = run(None)
        print(f"[bench] serving ({name}) saturation {sat['requests_per_s']:.0f} requests/s, "
              f"{sat['solves_per_s'] / 1e6:.0f} M solves/s", file=sys.stderr, flush=True)
        if rates is None:
            rates = [f * sat["requests_per_s"] for f in args.serve_load]
        results = []
        for f, rate in zip(args.serve_load, rates):
            r = run(rate)
            r["load"] = f
            # arrivals faster than this design completes: the queue grows for the
            # whole run, and the latencies measure the run's length
            r["overloaded"] = rate > sat["requests_per_s"]
            results.append(r)
            print(f"[bench] serving ({name}) at {rate:.0f}/s: p50 {r['p50_ms']:.2f} ms p99 "
                  f"{r['p99_ms']:.2f} ms, {r['solves_per_s'] / 1e6:.0f} M solves/s",
                  file=sys.stderr, flush=True)
        for s in solvers.values():
            s.close()
        for q in pool:
            q.pop("out", None)
        return {"saturation": sat, "rates": results}, rates

    batched, rates = design(rt.RT_SERVE_BATCHED, None, args.serve_requests)
    # the persistent worker saturates an order of magnitude lower: a quarter of
    # the requests per run keeps the line's run time bounded
    persistent, _ = design(rt.RT_SERVE_PERSISTENT, rates, max(100, args.serve_requests // 4))
    persistent["requests_per_run"] = max(100, args.serve_requests // 4)
    out = {"pool": len(pool),
           "mix": "columns U{1..4096}, layers U{20..120}, bins {30,100,300}, cloud fraction "
                  "U[0,0.5], half FP64 / half mixed",
           "requests_per_run": args.serve_requests,
           "rates_from": "fractions of the batched saturation rate, the same for both designs"}
    out.update(batched)
    out["serve_mode"] = "batched"
    out["persistent"] = persistent
    return out


def high_resolution(args, torch, rt, synth) -> tuple[dict, dict]:
    """The 10242 x 80 x 300 workload (FP64 and mixed, the kernel and tile the
    library picks): time per solve and the HBM roofline fraction."""
    work = synth.make("cfg4")
    C, N, NB = work["n_cols"], work["n_layers"], work["n_bins"]
    s = rt.Solver(work["lambda_edges"], work["F_star"])
    inp = rt.to_device(work)
    sample = column_subset(work, np.arange(0, C, 100))   # 1 % of the columns, for the CPU oracle
    del work
    copy_gbs = copy_bandwidth(torch)
    out = s.outputs(C, N)
    steps = max(3, min(args.steps, 10))
    res = {"workload": WORKLOADS["cfg4"], "n_cols": C, "n_layers": N, "n_bins": NB,
           "steps": steps}
    abytes = algorithmic_bytes(C, N, NB)
    for prec, tag in ((rt.RT_FP64, "fp64"), (rt.RT_MIXED, "mixed")):
        kid = s.kernel_for(inp, out, prec)
        kname = KERNEL_NAMES[kid] + ("<true>" if prec == rt.RT_MIXED else "<false>")
        print(f"[bench] cfg4 {tag} ({kname})", file=sys.stderr, flush=True)
        _, tot, per = time_path(s, inp, out, prec, steps, 2, torch)
        ms = tot / steps
        ach = abytes / (ms * 1e-3) / 1e9
        res[tag] = {"ms_per_step": ms, "value": C * NB / (ms * 1e-3), "kernel": kname,
                    "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                 "copy_gbs": copy_gbs, "frac_vs_copy": ach / copy_gbs,
                                 "algorithmic_bytes": abytes,
                                 "traffic": traffic_from_profiles(kname, "cfg4")}}
    s.close()
    del inp, out
    torch.cuda.empty_cache()
    return res, sample


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-runs", type=int, default=5,
                    help="whole oracle solves per CPU timing (median reported)")
    ap.add_argument("--workload", default="cfg1", choices=sorted(WORKLOADS))
    ap.add_argument("--kernel", default="auto", choices=sorted(KERNEL_IDS),
                    help="solve kernel of the headline line (auto: tuned choice)")
    ap.add_argument("--compare-kernels", action="store_true",
                    help="also time both kernels at their default tiles")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving mix")
    ap.add_argument("--no-cfg4", action="store_true",
                    help="skip the 10242 x 80 x 300 high-resolution solve")
    ap.add_argument("--serve-pool", type=int, default=16)
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-copies", type=int, default=4)
    ap.add_argument("--serve-budget-gib", type=int, default=32)
    ap.add_argument("--serve-load", type=float, nargs="+", default=[0.5, 0.8],
                    help="Poisson arrival rates as fractions of the measured saturation")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run 5 device-to-device copies of this many bytes (calibrates "
                         "the HBM byte counters against a kernel of known traffic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solve has no "
              "cross-GPU step; columns shard across GPUs without communication.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_02293_amd import rt, synth

    if args.copy_bytes:
        n = args.copy_bytes // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "read": n * 8, "written": n * 8}))
        return

    WORKLOAD = args.workload
    pre = None
    if WORKLOAD == "cfg1_optics":
        atm = synth.make_atmosphere("cfg1")
        work = dict(atm, gauss_w=synth.gauss_points(20)[1], n_gauss=20, sublayer=True,
                    opacities=synth.opacity_table(atm["n_bins"], 20))
    elif WORKLOAD == "cfg1_kdist":
        work = synth.make_kdist("cfg1", n_gauss=20)
    elif WORKLOAD == "cfg1_sub":
        work = synth.make_sublayer("cfg1")
    else:
        work = synth.make(WORKLOAD)
    C, N = work["n_cols"], work["n_layers"]
    NB = work["n_bins"] * work.get("n_gauss", 1)      # solves per column
    s = rt.Solver(work["lambda_edges"], work["F_star"], gauss_weights=work.get("gauss_w"))
    if WORKLOAD == "cfg1_optics":
        s.set_opacities(work["opacities"])
        inp = {k: torch.from_numpy(np.ascontiguousarray(work[k])).cuda()
               for k in ("p_iface", "T_iface", "p_center", "T_center", "mu_star", "T_int")}
        opt = s.optical_properties(inp, sublayer=True)
        inp.update(opt)
        pre = lambda: s.optical_properties(inp, sublayer=True, out=opt)
    else:
        inp = rt.to_device(work)
    out = s.outputs(C, N, sublayer=work.get("sublayer", False))
    if work.get("sublayer"):
        N = 2 * N                                       # slabs
    torch.cuda.synchronize()
    print(f"[bench] {WORKLOAD} {C}x{N}x{NB} resident; timing FP64", file=sys.stderr, flush=True)

    kernel = KERNEL_IDS[args.kernel]
    # the kernel that runs, as the library resolves the request time_path makes
    kw = {} if kernel is None else {"kernel": kernel, "cols_per_block": 0}
    used = s.kernel_for(inp, out, rt.RT_FP64, **kw)
    used_m = s.kernel_for(inp, out, rt.RT_MIXED, **kw)
    kname, kname_m = KERNEL_NAMES[used] + "<false>", KERNEL_NAMES[used_m] + "<true>"
    wall, tot, per = time_path(s, inp, out, rt.RT_FP64, args.steps, args.warmup, torch, kernel,
                               pre)
    summed = ("F_up", "F_dn", "F_beam", "F_net", "heating")
    host = {"fp64": {k: out[k].cpu().numpy() for k in summed}}   # the last timed solve
    ms = tot / args.steps
    value = C * NB / (ms * 1e-3)
    abytes = algorithmic_bytes(C, N, NB)
    achieved = abytes / (ms * 1e-3) / 1e9
    traffic = traffic_from_profiles(kname) if WORKLOAD == "cfg1" else None
    copy_gbs = copy_bandwidth(torch)
    line = {
        "metric": METRIC, "value": value, "unit": "column·bin solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[WORKLOAD] + ", FP64",
                   "n_cols": C, "n_layers": N, "n_bins": NB, "precision": "fp64"},
        "latency_ms": {"p50": pct(per, 50), "p99": pct(per, 99)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "copy_gbs": copy_gbs, "frac_vs_copy": achieved / copy_gbs,
                     "traffic": traffic, "algorithmic_bytes": abytes,
                     "kernel": kname, "kernel_ms": ms},
    }
    if WORKLOAD == "cfg1":
        line["valu_issue"] = valu_issue(kname, ms)
        line["fp_rate"] = fp_rates(kname, ms)
    if not args.no_mixed:
        print("[bench] timing mixed", file=sys.stderr, flush=True)
        wall_m, tot_m, per_m = time_path(s, inp, out, rt.RT_MIXED, args.steps, args.warmup,
                                         torch, kernel, pre)
        ms_m = tot_m / args.steps
        host["mixed"] = {k: out[k].cpu().numpy() for k in summed}
        ach_m = abytes / (ms_m * 1e-3) / 1e9
        line["mixed"] = {"value": C * NB / (ms_m * 1e-3), "ms_per_step": ms_m,
                         "speedup_vs_fp64": ms / ms_m,
                         "latency_ms": {"p50": pct(per_m, 50), "p99": pct(per_m, 99)},
                         "roofline": {"bound": "hbm", "achieved": ach_m, "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": ach_m / HBM_PEAK_GBS,
                                      "copy_gbs": copy_gbs, "frac_vs_copy": ach_m / copy_gbs,
                                      "traffic": (traffic_from_profiles(kname_m)
                                                  if WORKLOAD == "cfg1" else None),
                                      "kernel": kname_m}}
        if WORKLOAD == "cfg1":
            line["mixed"]["valu_issue"] = valu_issue(kname_m, ms_m)
            line["mixed"]["fp_rate"] = fp_rates(kname_m, ms_m)
    if args.compare_kernels:
        cmp = {}
        for kid, kn in KERNEL_NAMES.items():
            for prec, tag in ((rt.RT_FP64, "fp64"), (rt.RT_MIXED, "mixed")):
                print(f"[bench] timing {kn} {tag}", file=sys.stderr, flush=True)
                _, t, _ = time_path(s, inp, out, prec, args.steps, args.warmup, torch, kid)
                cmp[f"{kn}:{tag}"] = t / args.steps
        line["kernels_ms"] = cmp
    s.close()
    del inp, out
    torch.cuda.empty_cache()
    default = WORKLOAD == "cfg1"
    if default and not args.no_serving:
        print("[bench] serving mix", file=sys.stderr, flush=True)
        line["serving"] = serving(args, torch, rt, synth)
        torch.cuda.empty_cache()
    cfg4_sample = None
    if default and not args.no_cfg4:
        line["cfg4"], cfg4_sample = high_resolution(args, torch, rt, synth)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        small = synth.make("cfg0") if default else None
        line["cpu_baseline"], ref = cpu_baseline(work, small, args.cpu_runs, cfg4_sample)
        if not work.get("sublayer") and work.get("n_gauss", 1) == 1:
            # the timed solves' errors against the oracle's result (all columns), and
            # against its binary128 build on every 10th column (the FP64 oracle's own
            # rounding reaches ~1e-10 of the gross flux at this shape)
            import oracle
            cols = np.arange(0, C, 10)
            wq = column_subset(work, cols)
            threads = line["cpu_baseline"]["cores"]
            refq = oracle.solve(wq, n_threads=threads, extended=True)
            line["error_vs_oracle"] = {
                "scale": "bin sums; F_up, F_dn, F_beam over max(|ref|, 1e-3 S), F_net over S, "
                         "heating as Q dp/g over S; S = the column's largest gross flux",
                "fp64_oracle_all_columns": {tag: error_stats(h, ref, work["p_iface"])
                                            for tag, h in host.items()},
                f"binary128_oracle_{cols.size}_columns": {
                    tag: error_stats({k: v[:, cols] for k, v in h.items()}, refq, wq["p_iface"])
                    for tag, h in host.items()}}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
