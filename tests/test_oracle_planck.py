"""Pins of the oracle's Planck bin integral (Section 2.2.1: B at interfaces;
F_BOA = pi B(T_int)).  References: 40-digit mpmath quadrature of the
definition in wavelength, the Stefan-Boltzmann law, and the Wien and
Rayleigh-Jeans limits."""
import math

import mpmath as mp
import numpy as np
import pytest

H, C, K = 6.62607015e-34, 299792458.0, 1.380649e-23
SIGMA = 2 * math.pi ** 5 * K ** 4 / (15 * H ** 3 * C ** 2)


@pytest.fixture(autouse=True, params=["fp64", "binary128"])
def build(request, orc):
    """Each pin runs against both builds of the oracle source."""
    with orc.extended_build(request.param == "binary128"):
        yield request.param


def planck_mp(T, l1, l2, pieces=64):
    """B_lambda integrated over [l1, l2] in wavelength, 40 digits, subdivided."""
    mp.mp.dps = 40
    T, l1, l2 = mp.mpf(T), mp.mpf(l1), mp.mpf(l2)
    h, c, k = mp.mpf("6.62607015e-34"), mp.mpf(299792458), mp.mpf("1.380649e-23")
    f = lambda lam: 2 * h * c ** 2 / lam ** 5 / mp.expm1(h * c / (lam * k * T))
    pts = [l1 + (l2 - l1) * i / pieces for i in range(pieces + 1)]
    return float(mp.quad(f, pts))


@pytest.mark.parametrize("T,l1,l2", [
    (1000.0, 1e-6, 2e-6), (700.0, 0.3e-6, 0.35e-6), (1800.0, 26e-6, 30e-6),
    (1500.0, 0.3e-6, 30e-6), (50.0, 20e-6, 30e-6), (2500.0, 2.0e-6, 2.05e-6),
    (100.0, 10e-6, 11e-6), (4400.0, 0.3e-6, 0.4e-6)])
def test_planck_bin_vs_mpmath(orc, T, l1, l2):
    ref = planck_mp(T, l1, l2)
    assert orc.planck_bin(T, l1, l2) == pytest.approx(ref, rel=2e-14)


@pytest.mark.parametrize("T", [100.0, 700.0, 1234.5, 2200.0, 4400.0])
def test_stefan_boltzmann_partition(orc, T):
    """Bins partitioning (0, inf) sum to sigma T^4 / pi (tails are < 1e-15)."""
    edges = np.logspace(-8.5, 1.0, 480)
    s = sum(orc.planck_bin(T, a, b) for a, b in zip(edges[:-1], edges[1:]))
    assert s == pytest.approx(SIGMA * T ** 4 / math.pi, rel=1e-13)


def test_wien_limit(orc):
    """x >> 1: B_lambda -> 2hc^2/lam^5 exp(-x); narrow bin ~ midpoint value."""
    T, lam, d = 300.0, 0.5e-6, 1e-12
    x = H * C / (lam * K * T)
    approx = 2 * H * C ** 2 / lam ** 5 * math.exp(-x) * d
    assert orc.planck_bin(T, lam - d / 2, lam + d / 2) == pytest.approx(approx, rel=1e-6)


def test_rayleigh_jeans_limit(orc):
    """x << 1: B_lambda -> 2 c k T / lam^4."""
    T, lam, d = 5000.0, 0.05, 1e-6
    approx = 2 * C * K * T / lam ** 4 * d
    assert orc.planck_bin(T, lam - d / 2, lam + d / 2) == pytest.approx(approx, rel=1e-4)


def test_zero_temperature(orc):
    assert orc.planck_bin(0.0, 1e-6, 2e-6) == 0.0
