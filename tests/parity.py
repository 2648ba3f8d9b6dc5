"""Shared helpers of the GPU parity tests: error metrics and sub-sampling.

Error metric (stated once, used everywhere).  Net fluxes cross zero, deep net
fluxes are a small fraction of the gross fluxes and cold short-wave bins
underflow, so each comparison is scaled by S, the largest gross flux
(F_up + F_dn + F_beam) of that column (bin-summed quantities) or of that
(column, bin) (per-bin quantities):
  F_up, F_dn, F_beam:  |x - x_ref| <= tol * max(|x_ref|, floor * S)
  F_net:               |x - x_ref| <= tol * S
  heating:             |Q - Q_ref| (p_j - p_{j+1}) / g <= tol * S
The reference is the oracle's extended-precision build (same code, binary128
arithmetic), whose own rounding error is far below these bars.  On the
sub-layer grid the centre fluxes are held to the same bars with the column's S.
"""
from __future__ import annotations

import numpy as np

GRAV = 47.0

# Relative tolerances and scale floors of the two paths (precision 0: FP64,
# 1: mixed).  Bin-summed fluxes use the floor 1e-6 S.  Per-bin fluxes: in FP64
# 1e-10 x 1e-6 S_cb would be below the unit roundoff of S_cb (2.2e-16), so the
# per-bin floor is 1e-5 S_cb (1e-15 S_cb absolute, a few ulp of S_cb); the
# mixed path's FP32 coefficients round at 6e-8 of each term, and its per-bin
# floor is 1e-3 S_cb.
TOL = {0: 1e-10, 1: 1e-5}
FLOOR = {0: 1e-6, 1: 1e-6}
FLOOR_BIN = {0: 1e-5, 1: 1e-3}


def subset(work: dict, cols) -> dict:
    """The same workload restricted to a list of columns (columns are independent)."""
    cols = np.asarray(cols)
    w = dict(work)
    w["n_cols"] = cols.size
    for k in ("p_iface", "T_iface", "T_center", "p_center"):
        if work.get(k) is not None:
            w[k] = np.ascontiguousarray(work[k][:, cols])
    for k in ("dtau", "w0", "g0"):
        w[k] = np.ascontiguousarray(work[k][:, cols, :])
    for k in ("mu_star", "T_int"):
        w[k] = np.ascontiguousarray(work[k][cols])
    if work.get("F_toa") is not None:
        w["F_toa"] = np.ascontiguousarray(work["F_toa"][cols])
    return w


def errors(out: dict, ref: dict, p_iface: np.ndarray, floor: float = 1e-3,
           cols=None, gravity: float = GRAV, floor_bin: float | None = None) -> dict:
    """Scaled errors of the bin-summed outputs (and per-bin ones if present)."""
    def host(x):
        return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)
    o = {k: host(v) for k, v in out.items()}
    if cols is not None:
        cols = np.asarray(cols)
        o = {k: (v[:, cols] if v.ndim == 2 and k not in ("F_up_toa_bin",) else
                 v[cols] if k in ("flags", "F_up_toa_bin") else
                 v[:, cols, :] if v.ndim == 3 else v) for k, v in o.items()}
    S = (ref["F_up"] + ref["F_dn"] + ref["F_beam"]).max(axis=0)
    e = {}
    for k in ("F_up", "F_dn", "F_beam"):
        e[k] = (np.abs(o[k] - ref[k]) / np.maximum(np.abs(ref[k]), floor * S)).max()
    e["F_net"] = (np.abs(o["F_net"] - ref["F_net"]) / S).max()
    if "F_up_center" in o and "F_up_center" in ref:
        for k in ("F_up_center", "F_dn_center", "F_beam_center"):
            e[k] = (np.abs(o[k] - ref[k]) / np.maximum(np.abs(ref[k]), floor * S)).max()
        e["F_net_center"] = (np.abs(o["F_net_center"] - ref["F_net_center"]) / S).max()
    dp = p_iface[:-1] - p_iface[1:]
    e["heating"] = (np.abs(o["heating"] - ref["heating"]) * dp / gravity / S).max()
    if "F_up_bin" in o and "F_up_bin" in ref:
        Sb = (ref["F_up_bin"] + ref["F_dn_bin"] + ref["F_beam_bin"]).max(axis=0)
        Sb = np.maximum(Sb, 1e-300)
        fb = floor if floor_bin is None else floor_bin
        for k in ("F_up_bin", "F_dn_bin"):
            e[k] = (np.abs(o[k] - ref[k]) / np.maximum(np.abs(ref[k]), fb * Sb)).max()
    if "F_up_toa_bin" in o and "F_up_toa_bin" in ref:
        Sb = (ref["F_up"] + ref["F_dn"] + ref["F_beam"]).max(axis=0)[:, None]
        e["F_up_toa_bin"] = (np.abs(o["F_up_toa_bin"] - ref["F_up_toa_bin"]) /
                             np.maximum(np.abs(ref["F_up_toa_bin"]), floor * Sb)).max()
    return e


def assert_close(out, ref, p_iface, tol, floor=1e-3, cols=None, keys=None, floor_bin=None):
    e = errors(out, ref, p_iface, floor=floor, cols=cols, floor_bin=floor_bin)
    bad = {k: v for k, v in e.items() if (keys is None or k in keys) and not (v <= tol)}
    assert not bad, f"errors above {tol}: {bad} (all: {e})"
    return e
