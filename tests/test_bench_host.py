"""Host-side pieces of bench.py: the oracle leg and the error statistics it
reports beside the throughput (no GPU)."""
import numpy as np

import bench
from paper_2203_02293_amd import synth


def test_cpu_baseline_returns_timing_and_outputs():
    w = synth.make("cfg0")
    small = bench.column_subset(w, np.arange(0, w["n_cols"], 8))
    t, ref = bench.cpu_baseline(w, small, runs=2)
    assert t["kind"] == "oracle" and t["value"] > 0 and t["cores"] >= 1
    # single-thread and all-thread medians on both workloads
    for tag in ("small", "workload"):
        runs = t["runs"][tag]
        for nt in {1, t["cores"]}:
            r = runs[f"{nt}_threads"]
            assert len(r["runs_s"]) == 2 and r["median_s"] == np.median(r["runs_s"])
    assert t["value"] == t["runs"]["workload"][f"{t['cores']}_threads"]["value"]
    C, N = w["n_cols"], w["n_layers"]
    assert ref["F_net"].shape == (N + 1, C) and ref["heating"].shape == (N, C)
    np.testing.assert_array_equal(ref["F_net"], ref["F_up"] - ref["F_dn"] - ref["F_beam"])


def test_error_stats_scaling():
    w = synth.make("cfg0")
    _, ref = bench.cpu_baseline(w, None, runs=1)
    keys = ("F_up", "F_dn", "F_beam", "F_net", "heating")
    same = bench.error_stats({k: ref[k].copy() for k in keys}, ref, w["p_iface"])
    assert all(v == 0.0 for d in same.values() for v in d.values())
    # one net flux off by 1e-7 of its column's largest gross flux
    got = {k: ref[k].copy() for k in keys}
    S = (ref["F_up"] + ref["F_dn"] + ref["F_beam"]).max(axis=0)
    got["F_net"][3, 5] += 1e-7 * S[5]
    e = bench.error_stats(got, ref, w["p_iface"])
    assert abs(e["F_net"]["max"] - 1e-7) < 1e-12 and e["F_net"]["median"] == 0.0
    # a heating error dQ in layer j is scaled by dp_j / g / S
    got = {k: ref[k].copy() for k in keys}
    dp = w["p_iface"][2, 7] - w["p_iface"][3, 7]
    got["heating"][2, 7] += 1e-6 * S[7] * 47.0 / dp
    e = bench.error_stats(got, ref, w["p_iface"])
    assert abs(e["heating"]["max"] - 1e-6) < 1e-12


def test_column_subset_matches_whole_solve():
    import oracle
    w = synth.make("cfg0")
    cols = np.arange(0, w["n_cols"], 10)
    whole = oracle.solve(w)
    part = oracle.solve(bench.column_subset(w, cols))
    for k in ("F_up", "F_dn", "F_net", "heating"):
        np.testing.assert_array_equal(part[k], whole[k][:, cols])
