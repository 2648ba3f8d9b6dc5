"""Pins of the oracle's k-distribution bins (Section 2.1.3: NB bins of NG
Gaussian points each, bin sums weighted by the quadrature weights)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2203_02293_amd import synth


def small(C=3, N=5, NB=4, seed=17):
    return synth.make(synth.Spec(name="k", g_level=1, n_layers=N, n_bins=NB, cloud="night",
                                 seed=seed), n_cols=C)


@pytest.mark.parametrize("ng", [1, 3, 20])
def test_identical_g_points_reduce_to_the_bin(ng):
    """Every g-point of a bin with the bin's own properties, weights summing to
    1: the weighted sums are the plain per-bin solve."""
    w = small()
    ref = O.solve(w, per_bin=True)
    _, gw = synth.gauss_points(ng)
    wk = dict(w, gauss_w=gw)
    for k in ("dtau", "w0", "g0"):
        wk[k] = np.ascontiguousarray(np.repeat(w[k], ng, axis=2))
    out = O.solve(wk, per_bin=True)
    S = (ref["F_up"] + ref["F_dn"] + ref["F_beam"]).max(axis=0)
    for k in ("F_up", "F_dn", "F_beam", "F_net"):
        assert np.max(np.abs(out[k] - ref[k]) / S) < 1e-14, k
    np.testing.assert_allclose(out["F_up_toa_bin"], ref["F_up_toa_bin"], rtol=1e-14)
    np.testing.assert_array_equal(out["F_up_bin"][:, :, ::ng], ref["F_up_bin"])
    np.testing.assert_array_equal(out["flags"], ref["flags"])


@pytest.mark.parametrize("a", [0.3, 2.0, 7.0])
def test_band_beam_matches_closed_form(a):
    """Beam through an absorbing band whose sorted opacity is linear in g,
    dtau(g) = a g, no emission: the band-averaged beam at the BOA is
    mu F* int_0^1 e^{-a g / mu} dg = mu F* (1 - e^{-a/mu}) / (a/mu), which
    20 Gauss points reproduce to rounding."""
    ng = 20
    gx, gw = synth.gauss_points(ng)
    mu, Fs = 0.6, 1000.0
    w = small(C=1, N=1, NB=1)
    w.update(mu_star=np.array([mu]), F_star=np.array([Fs]), T_iface=np.full((2, 1), 1e-3),
             T_int=np.zeros(1), gauss_w=gw,
             dtau=(a * gx).reshape(1, 1, ng), w0=np.zeros((1, 1, ng)), g0=np.zeros((1, 1, ng)))
    out = O.solve(w, O.Options(e_tau=1e-30))
    x = a / mu
    expect = mu * Fs * (-math.expm1(-x)) / x
    assert out["F_beam"][0, 0] == pytest.approx(expect, rel=1e-13)
    assert out["F_beam"][1, 0] == pytest.approx(mu * Fs, rel=1e-15)


def test_kdist_workload_is_a_k_distribution():
    """The synthetic k-distribution: weights sum to 1, optical depth rises with
    g within every bin, albedo is scattering over extinction."""
    w = synth.make_kdist(synth.Spec(name="k", g_level=1, n_layers=4, n_bins=3, seed=5),
                         n_cols=2, n_gauss=8)
    assert abs(w["gauss_w"].sum() - 1.0) < 1e-15
    d = w["dtau"].reshape(4, 2, 3, 8)
    assert np.all(np.diff(d, axis=3) >= -1e-300)
    out = O.solve(w, per_bin=True)
    assert out["rc"] == 0 and out["F_up_bin"].shape == (5, 2, 24)
    S = (out["F_up"] + out["F_dn"] + out["F_beam"]).max(axis=0)
    gw = w["gauss_w"]
    wsum = (out["F_up_bin"].reshape(5, 2, 3, 8) * gw).sum(axis=(2, 3))
    assert np.max(np.abs(wsum - out["F_up"]) / S) < 1e-14
