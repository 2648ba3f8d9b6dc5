"""Pins of the oracle's sub-layer grid (non-isothermal layers split at their
centres, Section 2.2.1 and the grid figure): against the pure-absorption
formal solution on the interleaved levels, against the single-slab solve when
the split is exact, and the heating identity."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2203_02293_amd import synth
from tests.test_oracle_pins import formal_solution

PI = math.pi


def sub_workload(C=3, N=5, NB=2, seed=5, cloud="none"):
    spec = synth.Spec(name="s", g_level=1, n_layers=N, n_bins=NB, cloud=cloud, seed=seed,
                      dtau_lo=1e-3, dtau_hi=3.0)
    return synth.make_sublayer(spec, n_cols=C)


def level_T(w):
    N = w["n_layers"]
    T = np.empty((2 * N + 1, w["n_cols"]))
    T[0::2], T[1::2] = w["T_iface"], w["T_center"]
    return T


def test_pure_absorption_on_interleaved_levels():
    """w0 = 0: every interface and centre flux, per bin, equals the formal
    solution through the 2N sub-layers with B linear in tau inside each; the
    centre outputs are the odd levels."""
    w = sub_workload()
    w["w0"] = np.zeros_like(w["w0"])
    w["g0"] = np.zeros_like(w["g0"])
    out = O.solve_sublayer(w, O.Options(e_tau=1e-30), per_bin=True, extended=True)
    T = level_T(w)
    lam = w["lambda_edges"]
    C, NB = w["n_cols"], w["n_bins"]
    for c in range(C):
        su = sd = sb = 0.0
        for b in range(NB):
            B = [O.planck_bin(t, lam[b], lam[b + 1]) for t in T[:, c]]
            Fboa = PI * O.planck_bin(w["T_int"][c], lam[b], lam[b + 1])
            ru, rd, rb = formal_solution(B, w["dtau"][:, c, b], w["mu_star"][c], w["F_star"][b],
                                         Fboa, 0.0)
            S = np.max(ru + rd + rb)
            assert np.max(np.abs(out["F_up_bin"][:, c, b] - ru)) < 1e-12 * S
            assert np.max(np.abs(out["F_dn_bin"][:, c, b] - rd)) < 1e-12 * S
            su, sd, sb = su + ru, sd + rd, sb + rb
        S = np.max(su + sd + sb)
        np.testing.assert_allclose(out["F_up"][:, c], su[0::2], rtol=0, atol=1e-12 * S)
        np.testing.assert_allclose(out["F_up_center"][:, c], su[1::2], rtol=0, atol=1e-12 * S)
        np.testing.assert_allclose(out["F_dn_center"][:, c], sd[1::2], rtol=0, atol=1e-12 * S)
        np.testing.assert_allclose(out["F_beam_center"][:, c], sb[1::2], rtol=1e-13, atol=0)
        np.testing.assert_allclose(out["F_net_center"][:, c],
                                   su[1::2] - sd[1::2] - sb[1::2], rtol=0, atol=1e-12 * S)


def centre_T_for_mean_B(Ta, Tb, lam1, lam2):
    """Centre temperature whose bin radiance is the mean of the two interface
    values (bisection; B is increasing in T)."""
    target = 0.5 * (O.planck_bin(Ta, lam1, lam2) + O.planck_bin(Tb, lam1, lam2))
    lo, hi = min(Ta, Tb), max(Ta, Tb)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if O.planck_bin(mid, lam1, lam2) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("improved", [0, 1])
def test_exact_split_equals_single_slab(improved):
    """One bin; each layer split into halves of dtau/2 with its own w0, g0 and a
    centre temperature whose B is the interface mean: the Planck function is
    then the same linear function of tau as in the single slab, so the
    interface fluxes (and heating) must equal the plain N-layer solve."""
    w = synth.make(synth.Spec(name="t", g_level=1, n_layers=6, n_bins=1, cloud="night",
                              seed=9), n_cols=4)
    w["lambda_edges"] = np.array([3.0e-6, 3.3e-6])
    w["F_star"] = np.array([2.0e4])
    w["mu_star"] = np.array([0.8, 0.35, -0.2, 0.6])
    opts = O.Options(improved=improved, e_tau=1e-30)
    ref = O.solve(w, opts, extended=True)
    N, C = w["n_layers"], w["n_cols"]
    lam1, lam2 = w["lambda_edges"]
    Tc = np.array([[centre_T_for_mean_B(w["T_iface"][j, c], w["T_iface"][j + 1, c], lam1, lam2)
                    for c in range(C)] for j in range(N)])
    ws = dict(w)
    ws.update(T_center=Tc, p_center=np.sqrt(w["p_iface"][:-1] * w["p_iface"][1:]),
              dtau=np.repeat(w["dtau"], 2, axis=0) / 2, w0=np.repeat(w["w0"], 2, axis=0),
              g0=np.repeat(w["g0"], 2, axis=0))
    out = O.solve_sublayer(ws, opts, extended=True)
    S = np.max(ref["F_up"] + ref["F_dn"] + ref["F_beam"], axis=0)
    for k in ("F_up", "F_dn", "F_beam", "F_net"):
        assert np.max(np.abs(out[k] - ref[k]) / S) < 1e-11, k
    dp = w["p_iface"][:-1] - w["p_iface"][1:]
    assert np.max(np.abs(out["heating"] - ref["heating"]) * dp / 47.0 / S) < 1e-11
    np.testing.assert_array_equal(out["flags"], ref["flags"])


def test_heating_is_interface_based_and_telescopes():
    w = sub_workload(C=4, N=7, NB=3, cloud="night")
    out = O.solve_sublayer(w)
    p, pc = w["p_iface"], w["p_center"]
    g = 47.0
    # heating of layer j = mass-weighted mean of its two sub-layers' heating
    ql = g * (out["F_net"][:-1] - out["F_net_center"]) / (p[:-1] - pc)
    qu = g * (out["F_net_center"] - out["F_net"][1:]) / (pc - p[1:])
    mix = (ql * (p[:-1] - pc) + qu * (pc - p[1:])) / (p[:-1] - p[1:])
    scale = np.abs(out["heating"]).max()
    assert np.max(np.abs(mix - out["heating"])) < 1e-12 * scale
    tel = (out["heating"] * (p[:-1] - p[1:]) / g).sum(0)
    np.testing.assert_allclose(tel, out["F_net"][0] - out["F_net"][-1], rtol=1e-10,
                               atol=1e-12 * np.abs(out["F_up"]).max())
