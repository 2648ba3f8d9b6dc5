"""Plain FP64 CPU oracle of the improved two-stream flux solve (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  The oracle exists to check the GPU library: only
the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the GPU library and never
imports it.

The arithmetic lives in ``rt_oracle.c`` (each function cites the part of the
paper it follows: Deitrick et al., arXiv 2203.02293, Section 2.2 and
Appendix B).  This module only builds that file with gcc, marshals numpy
arrays and exposes:

  planck_bin(T, lam1, lam2)            bin-integrated Planck radiance
  efit(w0, g0, opts)                   E of Section 2.2.4
  layer_coeffs(dtau, w0, g0, mu, opts) Appendix B coefficients of one layer
  assemble(...)/block_thomas(...)      the block system of Section 2.2.2
  column_bin(...)                      one (column, bin) solve
  solve(work, opts, ...)               the whole problem (bin sums, heating)
"""
from __future__ import annotations

import contextlib
import ctypes as ct
import dataclasses
import os
import pathlib
import subprocess

import numpy as np

HERE = pathlib.Path(__file__).resolve().parent
SRC = HERE / "rt_oracle.c"
LIB = HERE / "liborc_rt.so"
LIB_X = HERE / "liborc_rt_q.so"    # same source, binary128 arithmetic

F_GUARD, F_ECLAMP, F_ETAU, F_EDOMAIN, F_INVALID, F_NONFIN = 1, 2, 4, 8, 16, 32


def build(force: bool = True) -> pathlib.Path:
    """Compile the oracle with gcc (no FMA contraction, OpenMP for timing).

    Two builds of the same source: FP64 (the oracle) and binary128 (used to
    measure the rounding error of FP64 evaluations; the parity reference)."""
    for out, extra in ((LIB, []), (LIB_X, ["-DORC_QUAD=1"])):
        newest = max(SRC.stat().st_mtime, SRC.with_suffix(".h").stat().st_mtime)
        if force or not out.exists() or out.stat().st_mtime < newest:
            tmp = out.with_suffix(".so.tmp")
            subprocess.run(
                ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                 "-shared", "-fopenmp", "-Wall", "-Wno-maybe-uninitialized", *extra, "-o", str(tmp),
                 str(SRC), "-lquadmath", "-lm"],
                check=True)
            os.replace(tmp, out)
    return LIB


class Opts(ct.Structure):
    _fields_ = [("improved", ct.c_int32), ("noniso", ct.c_int32), ("e_clamp", ct.c_int32),
                ("pad_", ct.c_int32), ("eps2", ct.c_double), ("e_tau", ct.c_double),
                ("g_guard", ct.c_double), ("gravity", ct.c_double), ("cp", ct.c_double)]


class Layer(ct.Structure):
    _fields_ = [(n, ct.c_double) for n in
                ("E", "zp", "zm", "Tr", "chi", "xi", "psi", "Pi", "Gp", "Gm", "D")] + \
               [("flags", ct.c_uint32)]


_dp = ct.POINTER(ct.c_double)
_up = ct.POINTER(ct.c_uint32)


class Problem(ct.Structure):
    _fields_ = [("n_cols", ct.c_int32), ("n_layers", ct.c_int32), ("n_bins", ct.c_int32),
                ("col_begin", ct.c_int32), ("col_end", ct.c_int32), ("n_gauss", ct.c_int32),
                ("pad_", ct.c_int32), ("gauss_w", _dp), ("lambda_edges", _dp), ("F_star", _dp), ("p_iface", _dp), ("T_iface", _dp),
                ("dtau", _dp), ("w0", _dp), ("g0", _dp), ("mu_star", _dp), ("T_int", _dp),
                ("F_toa", _dp), ("F_up", _dp), ("F_dn", _dp), ("F_beam", _dp), ("F_net", _dp),
                ("heating", _dp), ("dTdt", _dp), ("F_up_toa_bin", _dp), ("F_up_bin", _dp),
                ("F_dn_bin", _dp), ("F_beam_bin", _dp), ("flags", _up)]


class OpTable(ct.Structure):
    _fields_ = [("n_temp", ct.c_int32), ("n_press", ct.c_int32), ("n_bins", ct.c_int32),
                ("n_gauss", ct.c_int32), ("temp", _dp), ("log10p", _dp), ("kappa", _dp),
                ("sigma_gas", _dp), ("cloud_abs", _dp), ("cloud_scat", _dp), ("cloud_g0", _dp),
                ("f_cloud", ct.c_double), ("m_mean", ct.c_double), ("gravity", ct.c_double)]


@dataclasses.dataclass
class Options:
    """Solver switches (defaults: improved, non-isothermal, Table 3 values)."""

    improved: int = 1
    noniso: int = 1
    e_clamp: int = 1
    eps2: float = 2.0 / 3.0
    e_tau: float = 1.0e-4
    g_guard: float = 1.0e-5
    gravity: float = 47.0
    cp: float = 12436.0

    def c(self) -> Opts:
        return Opts(self.improved, self.noniso, self.e_clamp, 0, self.eps2, self.e_tau,
                    self.g_guard, self.gravity, self.cp)


_libs: dict = {}
# Which build the functions below use when they are not told: FP64 (the
# oracle) unless a test switches to the binary128 build with extended_build().
_default = {"extended": False}


def load(path) -> ct.CDLL:
    """Load a build of the oracle source and declare its C signatures."""
    L = ct.CDLL(str(path))
    _declare(L)
    return L


def lib(extended: bool | None = None) -> ct.CDLL:
    """The FP64 oracle library, or its binary128 build if ``extended``
    (None: the build selected by ``extended_build``, FP64 by default)."""
    if extended is None:
        extended = _default["extended"]
    path = LIB_X if extended else LIB
    if path not in _libs:
        newest = max(SRC.stat().st_mtime, SRC.with_suffix(".h").stat().st_mtime)
        if not path.exists() or path.stat().st_mtime < newest:
            build(force=True)
        _libs[path] = load(path)
    return _libs[path]


@contextlib.contextmanager
def extended_build(on: bool = True):
    """Within the block, calls that name no build use the binary128 one (so
    the same pin tests can run against both builds of the source)."""
    saved = _default["extended"]
    _default["extended"] = bool(on)
    try:
        yield
    finally:
        _default["extended"] = saved


def _declare(L: ct.CDLL) -> None:
    for f in ("orc_rayleigh_h2", "orc_rayleigh_he"):
        getattr(L, f).restype = ct.c_double
        getattr(L, f).argtypes = [ct.c_double]
    L.orc_rayleigh_bin.restype = ct.c_double
    L.orc_rayleigh_bin.argtypes = [ct.c_double] * 4
    L.orc_kappa_interp.restype = ct.c_double
    L.orc_kappa_interp.argtypes = [ct.c_void_p, ct.c_double, ct.c_double, ct.c_int]
    L.orc_optics_point.restype = None
    L.orc_optics_point.argtypes = [ct.c_void_p, ct.c_double, ct.c_double, ct.c_int,
                                   ct.c_void_p, ct.c_void_p, ct.c_void_p]
    L.orc_optics.restype = ct.c_int
    L.orc_optics.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.c_int] + [ct.c_void_p] * 7
    L.orc_planck_bin.restype = ct.c_double
    L.orc_planck_bin.argtypes = [ct.c_double, ct.c_double, ct.c_double]
    L.orc_efit.restype = ct.c_double
    L.orc_efit.argtypes = [ct.c_double, ct.c_double, ct.POINTER(Opts), _up]
    L.orc_layer_coeffs.restype = None
    L.orc_layer_coeffs.argtypes = [ct.c_double, ct.c_double, ct.c_double, ct.c_double,
                                   ct.POINTER(Opts), ct.POINTER(Layer)]
    L.orc_assemble.restype = ct.c_int
    L.orc_assemble.argtypes = [ct.c_int, _dp, _dp, _dp, _dp, ct.c_long, ct.c_double,
                               ct.c_double, ct.c_double, ct.c_double, ct.POINTER(Opts),
                               _dp, _dp, _dp, _dp, _dp, _up]
    L.orc_block_thomas.restype = ct.c_int
    L.orc_block_thomas.argtypes = [ct.c_int, _dp, _dp, _dp, _dp, _dp]
    L.orc_column_bin.restype = ct.c_int
    L.orc_column_bin.argtypes = [ct.c_int, _dp, _dp, _dp, _dp, ct.c_long, ct.c_double,
                                 ct.c_double, ct.c_double, ct.c_double, ct.POINTER(Opts),
                                 _dp, _dp, _dp, _up]
    L.orc_solve.restype = ct.c_int
    L.orc_solve.argtypes = [ct.POINTER(Problem), ct.POINTER(Opts), ct.c_int]
    L.orc_max_threads.restype = ct.c_int


def _p(a: np.ndarray | None):
    if a is None:
        return ct.cast(None, _dp)
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- scalar API
def planck_bin(T: float, lam1: float, lam2: float) -> float:
    return lib().orc_planck_bin(float(T), float(lam1), float(lam2))


def efit(w0: float, g0: float, opts: Options | None = None) -> tuple[float, int]:
    o = (opts or Options()).c()
    fl = ct.c_uint32(0)
    E = lib().orc_efit(float(w0), float(g0), ct.byref(o), ct.byref(fl))
    return E, fl.value


def layer_coeffs(dtau: float, w0: float, g0: float, mu: float,
                 opts: Options | None = None) -> dict:
    o = (opts or Options()).c()
    L = Layer()
    lib().orc_layer_coeffs(float(dtau), float(w0), float(g0), float(mu), ct.byref(o),
                           ct.byref(L))
    return {n: getattr(L, n) for n, _ in Layer._fields_}


# ------------------------------------------------------------ one (col, bin)
def assemble(B, dtau, w0, g0, mu, Fstar, F_boa=0.0, F_toa=0.0, opts: Options | None = None):
    """Block matrices of one (column, bin): A, B, C [N+1,2,2], D [N+1,2], beam [N+1]."""
    B, dtau, w0, g0 = map(_f64, (B, dtau, w0, g0))
    N = dtau.size
    A, Bm, Cm = (np.zeros((N + 1, 2, 2)) for _ in range(3))
    D, Fb = np.zeros((N + 1, 2)), np.zeros(N + 1)
    fl = ct.c_uint32(0)
    o = (opts or Options()).c()
    lib().orc_assemble(N, _p(B), _p(dtau), _p(w0), _p(g0), 1, float(mu), float(Fstar),
                       float(F_boa), float(F_toa), ct.byref(o), _p(A), _p(Bm), _p(Cm),
                       _p(D), _p(Fb), ct.byref(fl))
    return A, Bm, Cm, D, Fb, fl.value


def block_thomas(A, Bm, Cm, D) -> np.ndarray:
    A, Bm, Cm, D = map(_f64, (A, Bm, Cm, D))
    N = A.shape[0] - 1
    X = np.zeros((N + 1, 2))
    rc = lib().orc_block_thomas(N, _p(A), _p(Bm), _p(Cm), _p(D), _p(X))
    if rc:
        raise ArithmeticError("singular pivot block")
    return X


def column_bin(B, dtau, w0, g0, mu, Fstar, F_boa=0.0, F_toa=0.0,
               opts: Options | None = None):
    """Fluxes of one (column, bin) from interface Planck values B[N+1].

    Returns (F_up, F_dn, F_beam, flags), arrays over interfaces 0 (BOA)..N (TOA).
    """
    B, dtau, w0, g0 = map(_f64, (B, dtau, w0, g0))
    N = dtau.size
    fu, fd, fb = np.zeros(N + 1), np.zeros(N + 1), np.zeros(N + 1)
    fl = ct.c_uint32(0)
    o = (opts or Options()).c()
    rc = lib().orc_column_bin(N, _p(B), _p(dtau), _p(w0), _p(g0), 1, float(mu), float(Fstar),
                              float(F_boa), float(F_toa), ct.byref(o), _p(fu), _p(fd), _p(fb),
                              ct.byref(fl))
    if rc:
        raise ArithmeticError("singular pivot block")
    return fu, fd, fb, fl.value


# ----------------------------------------------------------------- problem
def solve(work: dict, opts: Options | None = None, per_bin: bool = False,
          cols: tuple[int, int] | None = None, n_threads: int = 0,
          F_toa: np.ndarray | None = None, extended: bool | None = None) -> dict:
    """Solve every (column, bin) of a workload dict (layouts as in ``synth``).

    ``cols`` restricts the solve to a column range (other outputs stay zero).
    ``n_threads`` = 0 uses OpenMP's default.  ``extended`` runs the same code
    in binary128 (parity reference; results rounded to FP64).  A k-distribution
    workload carries ``gauss_w`` [NG] (g-point weights of every bin, summing to
    1) and per-(bin, g-point) arrays of NB*NG entries; per-bin outputs are then
    per (bin, g-point) and ``F_up_toa_bin`` is the weighted sum over g.
    """
    C, N, NB = int(work["n_cols"]), int(work["n_layers"]), int(work["n_bins"])
    gw = work.get("gauss_w")
    NG = 1 if gw is None else int(np.asarray(gw).size)
    gw = None if gw is None else _f64(gw)
    c0, c1 = cols if cols is not None else (0, C)
    arr = {k: _f64(work[k]) for k in ("lambda_edges", "F_star", "p_iface", "T_iface",
                                        "dtau", "w0", "g0", "mu_star", "T_int")}
    Ft = None if F_toa is None else _f64(F_toa)
    out = {k: np.zeros((N + 1, C)) for k in ("F_up", "F_dn", "F_beam", "F_net")}
    out["heating"] = np.zeros((N, C))
    out["dTdt"] = np.zeros((N, C))
    out["F_up_toa_bin"] = np.zeros((C, NB))
    out["flags"] = np.zeros(C, dtype=np.uint32)
    if per_bin:
        for k in ("F_up_bin", "F_dn_bin", "F_beam_bin"):
            out[k] = np.zeros((N + 1, C, NB * NG))
    P = Problem(C, N, NB, c0, c1, NG, 0, _p(gw), _p(arr["lambda_edges"]), _p(arr["F_star"]),
                _p(arr["p_iface"]), _p(arr["T_iface"]), _p(arr["dtau"]), _p(arr["w0"]),
                _p(arr["g0"]), _p(arr["mu_star"]), _p(arr["T_int"]), _p(Ft),
                _p(out["F_up"]), _p(out["F_dn"]), _p(out["F_beam"]), _p(out["F_net"]),
                _p(out["heating"]), _p(out["dTdt"]), _p(out["F_up_toa_bin"]),
                _p(out.get("F_up_bin")), _p(out.get("F_dn_bin")), _p(out.get("F_beam_bin")),
                out["flags"].ctypes.data_as(_up))
    o = (opts or Options()).c()
    rc = lib(extended).orc_solve(ct.byref(P), ct.byref(o), int(n_threads))
    out["rc"] = rc
    return out


def solve_sublayer(work: dict, opts: Options | None = None, per_bin: bool = False,
                   cols: tuple[int, int] | None = None, n_threads: int = 0,
                   F_toa: np.ndarray | None = None, extended: bool | None = None) -> dict:
    """Sub-layer grid of non-isothermal layers (Section 2.2.1 and the grid
    figure): layer j is split at its centre into a lower sub-layer (interface j
    to centre j) and an upper one (centre j to interface j+1).  Each sub-layer
    is a slab with its own optical properties (``dtau``, ``w0``, ``g0`` of shape
    [2N][C][NB], slab 2j lower, 2j+1 upper) and a Planck function linear in
    optical depth between its two boundary levels, which is what the four
    sub-layer flux relations of Section 2.2.1 state.  So the system is the
    plain one over 2N slabs whose levels alternate interface, centre,
    interface, ...; interface fluxes are the even levels, centre fluxes the odd
    ones, and the heating of layer j comes from its interface net fluxes and
    pressures (Section 2.2.5).  ``work`` holds ``T_center`` and ``p_center``
    [N][C] besides the usual arrays; ``n_layers`` counts layers, not slabs.
    """
    o = opts or Options()
    N, C = int(work["n_layers"]), int(work["n_cols"])
    Tl = np.empty((2 * N + 1, C))
    pl = np.empty((2 * N + 1, C))
    Tl[0::2], Tl[1::2] = _f64(work["T_iface"]), _f64(work["T_center"])
    pl[0::2], pl[1::2] = _f64(work["p_iface"]), _f64(work["p_center"])
    w2 = dict(work)
    w2.update(n_layers=2 * N, T_iface=Tl, p_iface=pl)
    r = solve(w2, o, per_bin, cols, n_threads, F_toa, extended)
    out = {}
    for k in ("F_up", "F_dn", "F_beam", "F_net"):
        out[k] = np.ascontiguousarray(r[k][0::2])
        out[k + "_center"] = np.ascontiguousarray(r[k][1::2])
    p = _f64(work["p_iface"])
    out["heating"] = o.gravity * (out["F_net"][:-1] - out["F_net"][1:]) / (p[:-1] - p[1:])
    out["dTdt"] = out["heating"] / o.cp
    out["F_up_toa_bin"] = r["F_up_toa_bin"]
    out["flags"] = r["flags"]   # the interleaved pressures must decrease: centres in between
    out["rc"] = r["rc"]
    if per_bin:
        for k in ("F_up_bin", "F_dn_bin", "F_beam_bin"):
            out[k] = r[k]        # all 2N+1 levels
    return out


# ----------------------------------------------------------------- optical properties
def rayleigh_h2(lam_m: float) -> float:
    return lib().orc_rayleigh_h2(float(lam_m))


def rayleigh_he(lam_m: float) -> float:
    return lib().orc_rayleigh_he(float(lam_m))


def rayleigh_bin(lam1: float, lam2: float, x_h2: float, x_he: float) -> float:
    return lib().orc_rayleigh_bin(float(lam1), float(lam2), float(x_h2), float(x_he))


class _Tab:
    """An opacity-table dict (layout of ``synth.opacity_table``) as the C struct;
    keeps the arrays alive."""

    def __init__(self, tab: dict, lambda_edges, gravity: float):
        lam = _f64(lambda_edges)
        NB = lam.size - 1
        self.arr = {k: _f64(tab[k]) for k in ("temp", "log10p", "kappa")}
        self.arr["sigma_gas"] = np.array([rayleigh_bin(lam[b], lam[b + 1], tab["x_h2"],
                                                       tab["x_he"]) for b in range(NB)])
        for k in ("cloud_abs", "cloud_scat", "cloud_g0"):
            self.arr[k] = None if tab.get(k) is None else _f64(tab[k])
        NG = int(tab.get("n_gauss", 1))
        self.c = OpTable(self.arr["temp"].size, self.arr["log10p"].size, NB, NG,
                         _p(self.arr["temp"]), _p(self.arr["log10p"]), _p(self.arr["kappa"]),
                         _p(self.arr["sigma_gas"]), _p(self.arr["cloud_abs"]),
                         _p(self.arr["cloud_scat"]), _p(self.arr["cloud_g0"]),
                         float(tab["f_cloud"]), float(tab["m_mean"]), float(gravity))


def kappa_interp(tab: dict, lambda_edges, T: float, p: float, bg: int) -> float:
    t = _Tab(tab, lambda_edges, 1.0)
    return lib().orc_kappa_interp(ct.byref(t.c), float(T), float(p), int(bg))


def optics_point(tab: dict, lambda_edges, T: float, p: float, bg: int) -> tuple:
    """(extinction per unit mass, w0, g0) at one (T, p) for (bin, g-point) bg."""
    t = _Tab(tab, lambda_edges, 1.0)
    ke, w, g = ct.c_double(), ct.c_double(), ct.c_double()
    lib().orc_optics_point(ct.byref(t.c), float(T), float(p), int(bg), ct.byref(ke),
                           ct.byref(w), ct.byref(g))
    return ke.value, w.value, g.value


def optics(work: dict, tab: dict, sublayer: bool = False, gravity: float = 47.0) -> dict:
    """dtau, w0, g0 of every slab from the opacity table (``work`` supplies
    T/p at interfaces and centres and the bin edges)."""
    t = _Tab(tab, work["lambda_edges"], gravity)
    C, N = int(work["n_cols"]), int(work["n_layers"])
    nbg = t.c.n_bins * t.c.n_gauss
    S = 2 * N if sublayer else N
    out = {k: np.zeros((S, C, nbg)) for k in ("dtau", "w0", "g0")}
    arr = {k: _f64(work[k]) for k in ("T_iface", "p_iface", "T_center", "p_center")}
    rc = lib().orc_optics(ct.byref(t.c), C, N, int(sublayer), _p(arr["T_iface"]),
                          _p(arr["p_iface"]), _p(arr["T_center"]), _p(arr["p_center"]),
                          _p(out["dtau"]), _p(out["w0"]), _p(out["g0"]))
    if rc:
        raise ValueError("bad optics arguments")
    return out


def max_threads() -> int:
    return lib().orc_max_threads()
