"""Seeded synthetic inputs for the improved two-stream solve.

This module only draws numbers: grid points, pressure and temperature
profiles, per-layer per-bin optical depth, single-scattering albedo and
asymmetry parameter, bin edges and a stellar spectrum.  It holds none of the
radiative-transfer arithmetic (no coefficients, no Planck bin integrals, no
solve) and is the one module that both the CPU oracle side and the GPU side
of the tests and benchmark draw their inputs from.

The shapes and value ranges stand in for the WASP-43b set-up of the paper
(icosahedral grid, 40 levels, 30 k-table bins; Sections 2.1.1, 2.1.3 and
4.2).  The real k-tables, chemistry, cloud optics and stellar template are
not available, so every array is synthetic; the recipe is fixed by a seed
(``numpy.random.Generator(PCG64)``, one stream per array).

Layouts (all C-contiguous float64):
  p_iface, T_iface : [N+1][C]   interface 0 = bottom of atmosphere (BOA)
  dtau, w0, g0     : [N][C][NB] layer j lies between interfaces j and j+1
  mu_star          : [C]        cosine of the stellar zenith angle (<=0: night)
  T_int            : [C]        interior temperature for the bottom flux
  lambda_edges     : [NB+1]     metres, ascending
  F_star           : [NB]       stellar flux at TOA, W m^-2, per bin
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np

BAR = 1.0e5  # Pa

# SI 2019 constants used only to shape the synthetic stellar spectrum.
_H = 6.62607015e-34
_C = 299792458.0
_K = 1.380649e-23


# --------------------------------------------------------------------------
# grid
# --------------------------------------------------------------------------
@functools.lru_cache(maxsize=8)
def icosahedral_points(g_level: int) -> tuple[np.ndarray, np.ndarray]:
    """Vertices of a recursively bisected icosahedron on the unit sphere.

    Returns (lat, lon) in radians; there are 10*4**g_level + 2 points
    (162 / 2562 / 10242 for g_level 2 / 4 / 5, the grids of Section 2.1.1).
    """
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    verts = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            verts += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(verts, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # faces: triples of mutually adjacent vertices (edge = minimal distance)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    edge = d[d > 1e-9].min()
    adj = np.abs(d - edge) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    assert len(faces) == 20
    pts = [tuple(p) for p in v]
    for _ in range(g_level):
        cache: dict[tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            if key not in cache:
                m = np.add(pts[i], pts[j])
                m /= np.linalg.norm(m)
                cache[key] = len(pts)
                pts.append(tuple(m))
            return cache[key]

        new_faces = []
        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    xyz = np.array(pts)
    assert xyz.shape[0] == 10 * 4 ** g_level + 2
    lat = np.arcsin(np.clip(xyz[:, 2], -1.0, 1.0))
    lon = np.arctan2(xyz[:, 1], xyz[:, 0])
    return lat, lon


# --------------------------------------------------------------------------
# workload description
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Spec:
    """Recipe of one synthetic workload (sizes and value distributions)."""

    name: str
    g_level: int = 4            # icosahedral refinement -> columns
    n_cols: int | None = None   # explicit column count (first n points)
    col_offset: int = 0         # index of the first icosahedral point used
    n_layers: int = 40
    n_bins: int = 30
    lam_min_um: float = 0.3
    lam_max_um: float = 30.0
    p_bot_bar: float = 100.0
    p_top_bar: float = 1.0e-6
    t_base: float = 700.0
    t_day: float = 1100.0
    t_noise: float = 20.0
    dtau_lo: float = 1.0e-6
    dtau_hi: float = 1.0e2
    w0_lo: float = 0.0
    w0_hi: float = 0.3
    cloud: str = "none"         # "none" | "night" | "fraction"
    cloud_fraction: float = 0.0
    cloud_p_lo_bar: float = 1.0e-3
    cloud_p_hi_bar: float = 1.0e-1
    cloud_w0_lo: float = 0.9
    cloud_w0_hi: float = 0.999
    cloud_g0_lo: float = 0.5
    cloud_g0_hi: float = 0.95
    t_star: float = 4400.0
    f_bol: float = 9.0e5
    t_int: float = 100.0
    seed: int = 1000


#: The paper-shaped workloads.  cfg1 is the GCM size of Section 4.2
#: (2562 columns x 40 levels x 30 bins); cfg2 reuses cfg1's inputs.
SPECS: dict[str, Spec] = {
    "cfg0": Spec(name="cfg0", g_level=2, seed=1000),
    "cfg1": Spec(name="cfg1", g_level=4, cloud="night", seed=1001),
    "cfg4": Spec(name="cfg4", g_level=5, n_layers=80, n_bins=300, dtau_lo=1e-8,
                 dtau_hi=1e3, cloud="night", cloud_w0_hi=0.9999,
                 cloud_g0_hi=0.98, seed=1004),
}
SPECS["cfg2"] = dataclasses.replace(SPECS["cfg1"], name="cfg2")
#: Few deep columns (the grids that split columns into layer segments): one
#: dayside column (mu_star 0.85) of 4096 layers; 16 columns of 1000 layers at
#: the first icosahedral points (day and night), about half with cloud decks.
SPECS["deep1"] = Spec(name="deep1", g_level=4, n_cols=1, col_offset=5, n_layers=4096,
                      cloud="fraction", cloud_fraction=0.5, seed=1005)
SPECS["deep16"] = Spec(name="deep16", g_level=4, n_cols=16, n_layers=1000, cloud="fraction",
                       cloud_fraction=0.5, seed=1006)


def stellar_spectrum(lam_edges: np.ndarray, t_star: float, f_bol: float) -> np.ndarray:
    """Synthetic per-bin stellar flux at TOA (W m^-2), stand-in for the stellar template.

    Each bin holds the blackbody share of ``f_bol`` estimated by the spectral
    density at the bin's geometric centre times its width.  This is input data
    only; the solver takes the per-bin vector as given.
    """
    lo, hi = lam_edges[:-1], lam_edges[1:]
    lam = np.sqrt(lo * hi)
    x = _H * _C / (lam * _K * t_star)
    spec_density = 2.0 * _H * _C ** 2 / lam ** 5 / np.expm1(x)   # W m^-3 sr^-1
    sigma = 2.0 * math.pi ** 5 * _K ** 4 / (15.0 * _H ** 3 * _C ** 2)
    return f_bol * math.pi * spec_density * (hi - lo) / (sigma * t_star ** 4)


def _streams(seed: int, n: int) -> list[np.random.Generator]:
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(seed).spawn(n)]


def columns_from_points(lat: np.ndarray, lon: np.ndarray) -> np.ndarray:
    """Cosine of the stellar zenith angle, substellar point at (0, 0)."""
    return np.cos(lat) * np.cos(lon)


def make(spec: Spec | str, n_cols: int | None = None, mu_star: np.ndarray | None = None,
         seed: int | None = None) -> dict:
    """Draw one workload.  Returns a dict of numpy arrays plus ``spec``/sizes."""
    if isinstance(spec, str):
        spec = SPECS[spec]
    lat, lon = icosahedral_points(spec.g_level)
    mu_all = columns_from_points(lat, lon)
    C = n_cols if n_cols is not None else (spec.n_cols or mu_all.size)
    if mu_star is None:
        mu_all = np.roll(mu_all, -spec.col_offset)
        if C <= mu_all.size:
            mu = mu_all[:C].copy()
        else:
            mu = np.resize(mu_all, C)
    else:
        mu = np.asarray(mu_star, dtype=np.float64).copy()
        C = mu.size
    N, NB = spec.n_layers, spec.n_bins
    rs = _streams(spec.seed if seed is None else seed, 8)

    p1 = np.logspace(math.log10(spec.p_bot_bar * BAR), math.log10(spec.p_top_bar * BAR), N + 1)
    p_iface = np.repeat(p1[:, None], C, axis=1)
    T_iface = (spec.t_base + spec.t_day * np.maximum(mu, 0.0)[None, :] ** 0.25
               + spec.t_noise * rs[0].standard_normal((N + 1, C)))

    dp = p1[:-1] - p1[1:]
    scale = dp / dp.max()
    logu = rs[1].uniform(math.log(spec.dtau_lo), math.log(spec.dtau_hi), size=(N, C, NB))
    dtau = np.exp(logu) * scale[:, None, None]
    w0 = rs[2].uniform(spec.w0_lo, spec.w0_hi, size=(N, C, NB))
    g0 = np.zeros((N, C, NB))

    if spec.cloud != "none":
        if spec.cloud == "night":
            cloudy_col = mu <= 0.0
        else:
            cloudy_col = rs[3].uniform(size=C) < spec.cloud_fraction
        pm = np.sqrt(p1[:-1] * p1[1:])
        cloud_layer = (pm >= spec.cloud_p_lo_bar * BAR) & (pm <= spec.cloud_p_hi_bar * BAR)
        mask = cloud_layer[:, None] & cloudy_col[None, :]
        cw = rs[4].uniform(spec.cloud_w0_lo, spec.cloud_w0_hi, size=(N, C, NB))
        cg = rs[5].uniform(spec.cloud_g0_lo, spec.cloud_g0_hi, size=(N, C, NB))
        w0 = np.where(mask[:, :, None], cw, w0)
        g0 = np.where(mask[:, :, None], cg, g0)

    lam = np.logspace(math.log10(spec.lam_min_um), math.log10(spec.lam_max_um), NB + 1) * 1e-6
    return dict(
        spec=spec, n_cols=C, n_layers=N, n_bins=NB,
        p_iface=np.ascontiguousarray(p_iface), T_iface=np.ascontiguousarray(T_iface),
        dtau=np.ascontiguousarray(dtau), w0=np.ascontiguousarray(w0),
        g0=np.ascontiguousarray(g0), mu_star=mu,
        T_int=np.full(C, spec.t_int), lambda_edges=lam,
        F_star=stellar_spectrum(lam, spec.t_star, spec.f_bol),
    )


def make_sublayer(spec: Spec | str, n_cols: int | None = None, seed: int | None = None) -> dict:
    """Workload on the sub-layer grid of non-isothermal layers: T and p given at
    the layer centres (as a dynamical core supplies them, centre pressure the
    geometric mean of the interfaces), interface T linearly interpolated in
    log p between neighbouring centres and extrapolated at BOA and TOA.
    Per-level quantities (an opacity-like optical depth per unit pressure,
    albedo, asymmetry) are drawn at all 2N+1 levels, and each sub-layer takes
    the arithmetic mean of its two levels, as the paper prescribes for
    sub-layer properties.  dtau/w0/g0 have shape [2N][C][NB] (slab 2j = lower
    half of layer j)."""
    if isinstance(spec, str):
        spec = SPECS[spec]
    base = make(spec, n_cols=n_cols, seed=seed)
    C, N, NB = base["n_cols"], base["n_layers"], base["n_bins"]
    rs = _streams((spec.seed if seed is None else seed) + 7919, 4)
    p_if = base["p_iface"]
    p_c = np.sqrt(p_if[:-1] * p_if[1:])
    lp_if, lp_c = np.log(p_if[:, 0]), np.log(p_c[:, 0])
    mu = base["mu_star"]
    T_c = (spec.t_base + spec.t_day * np.maximum(mu, 0.0)[None, :] ** 0.25
           + spec.t_noise * rs[0].standard_normal((N, C)))
    T_if = np.empty((N + 1, C))
    for c in range(C):   # linear in log p through the centres, extended at the ends
        T_if[:, c] = np.interp(lp_if[::-1], lp_c[::-1], T_c[::-1, c])[::-1]
        if N > 1:
            sb = (T_c[0, c] - T_c[1, c]) / (lp_c[0] - lp_c[1])
            st = (T_c[-1, c] - T_c[-2, c]) / (lp_c[-1] - lp_c[-2])
            T_if[0, c] = T_c[0, c] + sb * (lp_if[0] - lp_c[0])
            T_if[-1, c] = T_c[-1, c] + st * (lp_if[-1] - lp_c[-1])
    T_if = np.maximum(T_if, 10.0)
    # levels 0..2N alternate interface, centre; sub-layer k lies between levels k and k+1
    p_lev = np.empty(2 * N + 1)
    p_lev[0::2], p_lev[1::2] = p_if[:, 0], p_c[:, 0]
    dp_sub = p_lev[:-1] - p_lev[1:]
    scale = dp_sub / (2.0 * dp_sub.max())
    k_lev = np.exp(rs[1].uniform(math.log(spec.dtau_lo), math.log(spec.dtau_hi),
                                 size=(2 * N + 1, C, NB)))
    w_lev = rs[2].uniform(spec.w0_lo, spec.w0_hi, size=(2 * N + 1, C, NB))
    g_lev = np.zeros((2 * N + 1, C, NB))
    if spec.cloud != "none":
        cloudy_col = mu <= 0.0 if spec.cloud == "night" else \
            rs[3].uniform(size=C) < spec.cloud_fraction
        cloud_lev = (p_lev >= spec.cloud_p_lo_bar * BAR) & (p_lev <= spec.cloud_p_hi_bar * BAR)
        mask = cloud_lev[:, None] & cloudy_col[None, :]
        cw = rs[3].uniform(spec.cloud_w0_lo, spec.cloud_w0_hi, size=(2 * N + 1, C, NB))
        cg = rs[3].uniform(spec.cloud_g0_lo, spec.cloud_g0_hi, size=(2 * N + 1, C, NB))
        w_lev = np.where(mask[:, :, None], cw, w_lev)
        g_lev = np.where(mask[:, :, None], cg, g_lev)
    mean = lambda a: 0.5 * (a[:-1] + a[1:])   # sub-layer value: mean of its two levels
    base.update(
        T_iface=np.ascontiguousarray(T_if), T_center=np.ascontiguousarray(T_c),
        p_center=np.ascontiguousarray(p_c),
        dtau=np.ascontiguousarray(mean(k_lev) * scale[:, None, None]),
        w0=np.ascontiguousarray(mean(w_lev)), g0=np.ascontiguousarray(mean(g_lev)),
        sublayer=True)
    return base


def gauss_points(n_gauss: int) -> tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre nodes and weights on [0, 1] (weights sum to 1): the
    quadrature over the cumulative variable g of a k-distribution bin."""
    x, w = np.polynomial.legendre.leggauss(n_gauss)
    return 0.5 * (x + 1.0), 0.5 * w


def make_kdist(spec: Spec | str, n_cols: int | None = None, n_gauss: int = 20,
               seed: int | None = None) -> dict:
    """Workload with k-distribution bins (Section 2.1.3: opacities sorted within
    each bin and sampled at n_gauss Gaussian points).  Per (layer, column, bin)
    the base recipe gives an optical depth; it is split into an absorbing part
    whose sorted opacity rises across the bin, k(g) = k_mid exp(s (g - 1/2))
    with a spread s ~ U[0, 8] per bin, and a scattering part the same for all
    g.  w0 at each g-point is scattering over total extinction, as the mixing
    rule prescribes, and g0 is the base recipe's (cloud decks).  Arrays hold
    NB * n_gauss entries per column, index bin * n_gauss + g."""
    if isinstance(spec, str):
        spec = SPECS[spec]
    base = make(spec, n_cols=n_cols, seed=seed)
    N, C, NB = base["n_layers"], base["n_cols"], base["n_bins"]
    rs = _streams((spec.seed if seed is None else seed) + 104729, 2)
    gx, gw = gauss_points(n_gauss)
    spread = rs[0].uniform(0.0, 8.0, size=NB)
    shape = np.exp(spread[:, None] * (gx[None, :] - 0.5))          # [NB][NG]
    shape /= (shape * gw[None, :]).sum(axis=1, keepdims=True)        # mean 1 over g
    scat = base["dtau"] * base["w0"]                                  # [N][C][NB]
    absb = base["dtau"] - scat
    dtau = absb[..., None] * shape[None, None] + scat[..., None]      # [N][C][NB][NG]
    with np.errstate(invalid="ignore", divide="ignore"):
        w0 = np.where(dtau > 0, scat[..., None] / dtau, 0.0)
    w0 = np.clip(w0, 0.0, 1.0)
    g0 = np.repeat(base["g0"][..., None], n_gauss, axis=3)
    base.update(dtau=np.ascontiguousarray(dtau.reshape(N, C, NB * n_gauss)),
                w0=np.ascontiguousarray(w0.reshape(N, C, NB * n_gauss)),
                g0=np.ascontiguousarray(g0.reshape(N, C, NB * n_gauss)),
                gauss_w=gw, n_gauss=n_gauss)
    return base


AMU = 1.66053906660e-27   # kg


def opacity_table(n_bins: int, n_gauss: int = 1, seed: int = 2024, n_temp: int = 60,
                  n_press: int = 28) -> dict:
    """Synthetic pre-mixed k-table standing in for the opacity calculator's
    (Section 2.1.3): n_temp temperatures 50-3000 K, n_press pressures 1e-6 to
    1e3 bar equally spaced in log p, absorption opacity per unit mass for every
    (bin, Gaussian point), log-normal across bins, rising with g inside a bin,
    with power-law pressure broadening and an exponential temperature
    dependence.  Condensate cross sections of 1 um particles (geometric
    cross section pi r^2 scaled per bin), cloud-to-gas ratio 1e-17 and a mean
    molecular mass of 2.34 amu as in the paper's set-up; H2/He volume mixing
    ratios 0.85/0.15 for Rayleigh scattering."""
    r = np.random.Generator(np.random.PCG64(seed))
    temp = np.linspace(50.0, 3000.0, n_temp)
    log10p = np.linspace(math.log10(1e-6 * BAR), math.log10(1e3 * BAR), n_press)
    nbg = n_bins * n_gauss
    k_bin = np.exp(r.normal(math.log(1e-2), 2.5, size=n_bins))          # m^2 / kg
    spread = r.uniform(0.0, 8.0, size=n_bins)
    gx = gauss_points(n_gauss)[0] if n_gauss > 1 else np.array([0.5])
    k_bg = (k_bin[:, None] * np.exp(spread[:, None] * (gx[None, :] - 0.5))).reshape(nbg)
    alpha = r.uniform(0.2, 0.8, size=nbg)                               # pressure broadening
    beta = r.uniform(-1.0, 2.0, size=nbg)                               # temperature trend
    P = (10.0 ** log10p) / BAR
    kappa = (k_bg[None, None, :] * (P[:, None, None] / 1.0) ** alpha[None, None, :]
             * np.exp(beta[None, None, :] * (temp[None, :, None] - 1000.0) / 1000.0))
    rad = 1e-6
    geo = math.pi * rad * rad
    return dict(temp=temp, log10p=log10p, kappa=np.ascontiguousarray(kappa), n_gauss=n_gauss,
                cloud_abs=geo * r.uniform(0.1, 1.0, size=n_bins),
                cloud_scat=geo * r.uniform(1.0, 2.5, size=n_bins),
                cloud_g0=r.uniform(0.5, 0.9, size=n_bins),
                f_cloud=1e-17, m_mean=2.34 * AMU, x_h2=0.85, x_he=0.15)


def make_atmosphere(spec: Spec | str, n_cols: int | None = None, seed: int | None = None) -> dict:
    """Temperatures and pressures at interfaces and layer centres (no optical
    properties): the input of the optical-properties step.  Centre pressure is
    the geometric mean of the interfaces; interface T is linearly interpolated
    in log p between centres (the sub-layer recipe of ``make_sublayer``)."""
    w = make_sublayer(spec, n_cols=n_cols, seed=seed)
    for k in ("dtau", "w0", "g0"):
        w.pop(k)
    return w


# --------------------------------------------------------------------------
# serving mix (uneven requests, Poisson arrivals)
# --------------------------------------------------------------------------
def serving_requests(n_requests: int, seed: int = 1003, max_cols: int = 4096,
                     layers=(20, 120), bins=(30, 100, 300)) -> list[dict]:
    """Request shapes for the serving mix: columns U{1..max_cols}, layers
    U{layers}, bins drawn from ``bins``, cloud fraction U[0, 0.5]; the values
    follow the cfg1 generators."""
    r = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n_requests):
        out.append(dict(
            n_cols=int(r.integers(1, max_cols + 1)),
            n_layers=int(r.integers(layers[0], layers[1] + 1)),
            n_bins=int(r.choice(bins)),
            cloud_fraction=float(r.uniform(0.0, 0.5)),
            seed=int(seed * 1000 + k),
        ))
    return out


def make_request(shape: dict, precision: str = "fp64") -> dict:
    """Draw the arrays of one serving request described by ``shape``."""
    spec = dataclasses.replace(
        SPECS["cfg1"], name="serve", n_layers=shape["n_layers"], n_bins=shape["n_bins"],
        cloud="fraction", cloud_fraction=shape["cloud_fraction"], seed=shape["seed"])
    lat, lon = icosahedral_points(5)
    r = np.random.Generator(np.random.PCG64(shape["seed"]))
    idx = r.choice(lat.size, size=shape["n_cols"], replace=False)
    mu = columns_from_points(lat[idx], lon[idx])
    w = make(spec, mu_star=mu)
    w["precision"] = precision
    return w


def poisson_arrivals(n: int, rate_hz: float, seed: int = 77) -> np.ndarray:
    """Arrival times (s) of a Poisson process at ``rate_hz``."""
    r = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(r.exponential(1.0 / rate_hz, size=n))
