"""Pins of the oracle's optical-properties step (k-table interpolation,
Rayleigh scattering of Appendix C, gas/condensate mixing of Section 2.2.3)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle as O
from paper_2203_02293_amd import synth

PI = math.pi


def n_h2(lam):   # printed refractivity fit, lam in m
    lp = lam / 1e-6
    return 1.358e-4 * (1 + 7.52e-3 / lp ** 2) + 1


def n_he(lam):
    lp = lam / 1e-6
    return 1e-8 * (2283 + 1.8102e13 / (1.5342e10 - lp ** -2)) + 1


@pytest.mark.parametrize("lam", [0.3e-6, 0.55e-6, 2e-6, 30e-6])
def test_rayleigh_matches_textbook_gas_formula(lam):
    """For a dilute gas (n - 1 << 1) the Lorentz-Lorenz form reduces to the
    textbook sigma = 32 pi^3 (n - 1)^2 / (3 N^2 lam^4); the two agree to
    O(n - 1) (cross sections in m^2, N in m^-3)."""
    for fn, n_of, N in ((O.rayleigh_h2, n_h2, 2.68678e25), (O.rayleigh_he, n_he, 2.546899e25)):
        n = n_of(lam)
        textbook = 32 * PI ** 3 * (n - 1) ** 2 / (3 * N ** 2 * lam ** 4)
        assert fn(lam) == pytest.approx(textbook, rel=5 * (n - 1))


def test_rayleigh_bin_is_the_wavenumber_average():
    lam1, lam2, xh, xe = 0.4e-6, 0.9e-6, 0.85, 0.15
    f = lambda nu: xh * O.rayleigh_h2(1 / nu) + xe * O.rayleigh_he(1 / nu)
    ref = quad(f, 1 / lam2, 1 / lam1, epsabs=0, epsrel=1e-13)[0] / (1 / lam1 - 1 / lam2)
    assert O.rayleigh_bin(lam1, lam2, xh, xe) == pytest.approx(ref, rel=1e-12)


def table(kfun, NB=2, NG=1):
    temp = np.array([100.0, 400.0, 900.0, 2000.0])
    log10p = np.linspace(0.0, 7.0, 5)
    kap = np.array([[[kfun(T, x, bg) for bg in range(NB * NG)] for T in temp] for x in log10p])
    return dict(temp=temp, log10p=log10p, kappa=kap, n_gauss=NG, cloud_abs=None,
                cloud_scat=None, cloud_g0=None, f_cloud=0.0, m_mean=2.34 * synth.AMU,
                x_h2=0.0, x_he=0.0)


LAM = np.array([1e-6, 2e-6, 3e-6])


def test_kappa_is_bilinear_in_T_and_log_p():
    """Exact at the nodes, exact for any function bilinear in (T, log10 p),
    and held at the table's edge outside it."""
    f = lambda T, x, bg: 1e-3 * (1 + bg) * (2 + 0.5 * T / 1000) * (1 + 0.3 * x) + 1e-6 * T * x
    tb = table(f)
    r = np.random.Generator(np.random.PCG64(4))
    for _ in range(20):
        T, x, bg = r.uniform(100, 2000), r.uniform(0, 7), int(r.integers(0, 2))
        assert O.kappa_interp(tb, LAM, T, 10 ** x, bg) == pytest.approx(f(T, x, bg), rel=1e-13)
    assert O.kappa_interp(tb, LAM, 400.0, 10 ** 3.5, 1) == pytest.approx(f(400, 3.5, 1), rel=1e-14)
    assert O.kappa_interp(tb, LAM, 20.0, 10 ** 9.0, 0) == pytest.approx(f(100, 7.0, 0), rel=1e-14)
    # curvature in T is not reproduced between nodes: a plain bilinear rule
    g = lambda T, x, bg: (T / 1000) ** 2
    tq = table(g)
    mid = 0.5 * (400 + 900)
    assert O.kappa_interp(tq, LAM, mid, 10.0, 0) == pytest.approx(0.5 * (0.16 + 0.81), rel=1e-14)


def test_mixing_limits_and_identity():
    tb = table(lambda T, x, bg: 0.02)
    m = tb["m_mean"]
    # pure absorber: no gas scattering, no condensates
    ke, w, g = O.optics_point(tb, LAM, 700.0, 1e4, 0)
    assert ke == pytest.approx(0.02, rel=1e-15) and w == 0.0 and g == 0.0
    # gas Rayleigh only: conservative scattering, isotropic
    tr = dict(table(lambda T, x, bg: 0.0), x_h2=1.0)
    ke, w, g = O.optics_point(tr, LAM, 700.0, 1e4, 1)
    assert w == 1.0 and g == 0.0
    assert ke == pytest.approx(O.rayleigh_bin(LAM[1], LAM[2], 1.0, 0.0) / m, rel=1e-14)
    # condensates only: their own albedo and asymmetry
    tc = dict(table(lambda T, x, bg: 0.0), f_cloud=1e-17, cloud_abs=np.array([1e-12, 2e-12]),
              cloud_scat=np.array([3e-12, 1e-12]), cloud_g0=np.array([0.7, 0.6]))
    ke, w, g = O.optics_point(tc, LAM, 700.0, 1e4, 0)
    assert w == pytest.approx(0.75, rel=1e-15) and g == pytest.approx(0.7, rel=1e-15)
    # everything: scattering part of the extinction = gas + condensate scattering
    ta = dict(tc, kappa=table(lambda T, x, bg: 0.05)["kappa"], x_h2=0.85, x_he=0.15)
    ke, w, g = O.optics_point(ta, LAM, 700.0, 1e4, 1)
    sg = O.rayleigh_bin(LAM[1], LAM[2], 0.85, 0.15)
    assert w * ke * m == pytest.approx(sg + 1e-17 * 1e-12, rel=1e-13)
    assert g == pytest.approx(1e-17 * 1e-12 * 0.6 / (sg + 1e-17 * 1e-12), rel=1e-13)


def test_layer_and_sublayer_optical_depths():
    """Uniform opacity: dtau is extinction x pressure thickness / g, and the two
    sub-layers of a layer add up to the layer."""
    tb = table(lambda T, x, bg: 0.03 * (1 + bg))
    w = synth.make_atmosphere(synth.Spec(name="a", g_level=1, n_layers=4, n_bins=2, seed=3),
                              n_cols=3)
    w["lambda_edges"] = LAM
    lay = O.optics(w, tb, sublayer=False)
    sub = O.optics(w, tb, sublayer=True)
    dp = w["p_iface"][:-1] - w["p_iface"][1:]
    np.testing.assert_allclose(lay["dtau"][:, :, 1], 0.06 * dp / 47.0, rtol=1e-14)
    np.testing.assert_allclose(sub["dtau"][0::2] + sub["dtau"][1::2], lay["dtau"], rtol=1e-13)
    assert np.all(sub["w0"] == 0.0) and np.all(lay["w0"] == 0.0)


def test_sublayer_properties_are_level_means():
    tb = table(lambda T, x, bg: 1e-3 * (T / 100) * (1 + x))
    tb.update(x_h2=0.85, x_he=0.15, f_cloud=1e-17, cloud_abs=np.array([1e-12, 1e-12]),
              cloud_scat=np.array([2e-12, 3e-12]), cloud_g0=np.array([0.8, 0.5]))
    w = synth.make_atmosphere(synth.Spec(name="a", g_level=1, n_layers=3, n_bins=2, seed=8),
                              n_cols=2)
    w["lambda_edges"] = LAM
    sub = O.optics(w, tb, sublayer=True)
    c, bg, j = 1, 1, 2
    lo = O.optics_point(tb, LAM, w["T_iface"][j, c], w["p_iface"][j, c], bg)
    ce = O.optics_point(tb, LAM, w["T_center"][j, c], w["p_center"][j, c], bg)
    dp = w["p_iface"][j, c] - w["p_center"][j, c]
    assert sub["dtau"][2 * j, c, bg] == pytest.approx(0.5 * (lo[0] + ce[0]) * dp / 47.0, rel=1e-14)
    assert sub["w0"][2 * j, c, bg] == pytest.approx(0.5 * (lo[1] + ce[1]), rel=1e-14)
    assert sub["g0"][2 * j, c, bg] == pytest.approx(0.5 * (lo[2] + ce[2]), rel=1e-14)


def test_opacity_table_workload_solves():
    """The synthetic k-table feeds a whole solve: optics then fluxes."""
    NB, NG = 4, 3
    tb = synth.opacity_table(NB, NG)
    w = synth.make_atmosphere(synth.Spec(name="a", g_level=1, n_layers=6, n_bins=NB, seed=2),
                              n_cols=3)
    opt = O.optics(w, tb, sublayer=True)
    assert np.all(opt["dtau"] > 0) and np.all((opt["w0"] >= 0) & (opt["w0"] <= 1))
    ws = dict(w, gauss_w=synth.gauss_points(NG)[1], **opt)
    out = O.solve_sublayer(ws)
    assert out["rc"] == 0 and np.all(np.isfinite(out["F_net"]))
