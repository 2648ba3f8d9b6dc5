"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

FP64 path: <= 1e-10 and mixed path: <= 1e-5 in the scaled metric of
``tests/parity.py``, against the oracle's extended-precision build.  Flags
(guard hits, E clamps, e_tau fallbacks, invalid inputs) must match exactly:
both sides take those decisions on the same FP64 values.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2203_02293_amd import synth
from tests.parity import FLOOR, FLOOR_BIN, TOL, assert_close, errors, subset

pytestmark = pytest.mark.gpu

FP64_TOL, MIXED_TOL = TOL[0], TOL[1]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def rt(torch):
    from paper_2203_02293_amd import rt as r
    r.lib()
    return r


KERNELS = [1, 2, 3]            # RT_KERNEL_LANE, RT_KERNEL_LAYER, RT_KERNEL_DEEP
KERNEL_IDS = ["lane", "layer", "deep"]


def gpu_solve(rt, torch, w, precision, per_bin=False, opts=None, F_toa=None, kernel=None,
              cols_per_block=None):
    o = opts or O.Options()
    s = rt.Solver(w["lambda_edges"], w["F_star"], improved=o.improved, noniso=o.noniso,
                  e_clamp=o.e_clamp, eps2=o.eps2, e_tau=o.e_tau, g_guard=o.g_guard,
                  gauss_weights=w.get("gauss_w"))
    inp = rt.to_device(w)
    if F_toa is not None:
        inp["F_toa"] = torch.from_numpy(np.ascontiguousarray(F_toa)).cuda()
    out = s.solve(inp, precision=precision, per_bin=per_bin, kernel=kernel,
                  cols_per_block=cols_per_block)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["flags"] = res["flags"].view(np.uint32)
    s.close()
    return res


def small(C, N, NB, seed, cloud="night", **kw):
    spec = synth.Spec(name="t", g_level=3, n_layers=N, n_bins=NB, cloud=cloud, seed=seed, **kw)
    return synth.make(spec, n_cols=C)


CASES = [
    ("ragged", dict(C=37, N=9, NB=7, seed=11)),
    ("bins30", dict(C=19, N=17, NB=30, seed=12)),
    ("one_col", dict(C=1, N=5, NB=3, seed=13)),
    ("one_bin", dict(C=300, N=4, NB=1, seed=14)),
    ("one_layer", dict(C=9, N=1, NB=5, seed=15)),
    ("wide_bins", dict(C=3, N=6, NB=300, seed=16)),
    ("deep", dict(C=4, N=120, NB=10, seed=17)),
    # bin-sum group widths 8 and 64 of the layer kernel's wavefront sums
    ("bins8", dict(C=21, N=7, NB=8, seed=18)),
    ("bins40", dict(C=13, N=9, NB=40, seed=19)),
]


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
@pytest.mark.parametrize("name,shape", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("mode", ["improved_noniso", "regular_noniso", "improved_iso"])
def test_small_fp64_and_mixed(rt, torch, name, shape, mode, kernel):
    print(f"\n[parity] {name} {shape} {mode} kernel={kernel}", flush=True)
    w = small(**shape)
    opts = O.Options(improved=int(mode.startswith("improved")), noniso=int("noniso" in mode))
    ref = O.solve(w, opts, per_bin=True, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, per_bin=True, opts=opts, kernel=kernel)
        e = assert_close(out, ref, w["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec])
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"], ref["flags"])


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_cfg0_full(rt, torch, kernel):
    w = synth.make("cfg0")
    print(f"\n[parity] cfg0 full {w['n_cols']}x{w['n_layers']}x{w['n_bins']} kernel={kernel}",
          flush=True)
    ref = O.solve(w, per_bin=True, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, per_bin=True, kernel=kernel)
        e = assert_close(out, ref, w["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec])
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"], ref["flags"])


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_cfg1_sampled(rt, torch, kernel):
    """GCM size 2562 x 40 x 30 solved whole on the GPU; 128 columns (day,
    night, cloud, terminator) checked against the oracle one by one."""
    w = synth.make("cfg1")
    print(f"\n[parity] cfg1 full {w['n_cols']}x{w['n_layers']}x{w['n_bins']} kernel={kernel}",
          flush=True)
    cols = np.unique(np.concatenate([np.linspace(0, w["n_cols"] - 1, 96).astype(int),
                                     np.argsort(np.abs(w["mu_star"]))[:32]]))
    ws = subset(w, cols)
    ref = O.solve(ws, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, kernel=kernel)
        e = assert_close(out, ref, ws["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec], cols=cols)
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"][cols], ref["flags"])


def test_default_tile_fits_lds(rt, torch):
    """2048 columns x 100 bins in FP64: the first default tile (7 columns of
    100 lanes) exceeds the LDS, so AUTO narrows it rather than failing."""
    w = small(C=2048, N=12, NB=100, seed=23)
    cols = np.linspace(0, 2047, 40).astype(int)
    ws = subset(w, cols)
    ref = O.solve(ws, extended=True)
    out = gpu_solve(rt, torch, w, rt.RT_FP64, kernel=0, cols_per_block=0)
    assert_close(out, ref, ws["p_iface"], FP64_TOL, floor=FLOOR[0], cols=cols)
    np.testing.assert_array_equal(out["flags"][cols], ref["flags"])


def test_toa_diffuse_flux(rt, torch):
    w = small(C=6, N=8, NB=5, seed=21)
    F_toa = np.random.Generator(np.random.PCG64(3)).uniform(0, 50, (6, 5))
    w["F_toa"] = F_toa
    ref = O.solve(w, per_bin=True, extended=True, F_toa=F_toa)
    out = gpu_solve(rt, torch, w, rt.RT_FP64, per_bin=True, F_toa=F_toa)
    assert_close(out, ref, w["p_iface"], FP64_TOL)


def edge_workload():
    """Columns built to sit on the paper's branch points."""
    w = small(C=11, N=6, NB=4, seed=31)
    w = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in w.items()}
    # w0 exactly at the 0.1 threshold and one ulp above it
    w["w0"][0, 0, :] = 0.1
    w["w0"][1, 0, :] = np.nextafter(0.1, 1.0)
    # dtau at e_tau and one ulp below, and exactly zero
    w["dtau"][2, 1, 0] = 1e-4
    w["dtau"][2, 1, 1] = np.nextafter(1e-4, 0.0)
    w["dtau"][3, 1, 2] = 0.0
    # very thick layer
    w["dtau"][4, 2, :] = 1e4
    # resonance: w0 = 0 (E = 1, lambda = 2) with mu = 0.5 -> D = 4 mu^2 - 1 = 0
    w["mu_star"][3] = 0.5
    w["w0"][:, 3, :] = 0.0
    # just outside the guard window
    w["mu_star"][4] = 0.5 + 3e-6
    w["w0"][:, 4, :] = 0.0
    # cloud with E fit below w0 (clamp region)
    w["w0"][:, 5, :] = 0.999
    w["g0"][:, 5, :] = 0.95
    # night column
    w["mu_star"][6] = -0.3
    # the terminator exactly (no beam) and a beam that is only just there
    w["mu_star"][8] = 0.0
    w["mu_star"][9] = 1e-300
    # a day column whose top layers are optically very thin (below and just
    # above e_tau): the beam sources of thin layers, where the printed forms
    # are differences of nearly equal terms
    w["mu_star"][10] = 0.7
    w["dtau"][5, 10, :] = 1e-12
    w["dtau"][4, 10, :] = 1e-6
    w["dtau"][3, 10, :] = 2e-4
    return w


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_edge_cases(rt, torch, kernel):
    w = edge_workload()
    ref = O.solve(w, per_bin=True, extended=True)
    assert ref["flags"][3] & O.F_GUARD and not ref["flags"][4] & O.F_GUARD
    assert ref["flags"][5] & O.F_ECLAMP and ref["flags"][1] & O.F_ETAU
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, per_bin=True, kernel=kernel)
        e = assert_close(out, ref, w["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec])
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"], ref["flags"])


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_mixed_fp32_input_storage(rt, torch, kernel):
    """input_dtype RT_F32: dtau, w0, g0 stored as floats on the mixed path.
    The oracle solves the same stored values (each float as the double it is)
    and the mixed bar applies; the flags match exactly, since the branch
    decisions see the stored floats.  The FP64 path refuses float inputs."""
    cases = [("cfg0", synth.make("cfg0")), ("edges", edge_workload()),
             ("deep", small(C=4, N=120, NB=10, seed=17)), ("bins300", small(C=3, N=6, NB=300, seed=16))]
    for name, w in cases:
        print(f"\n[parity] fp32 inputs {name} kernel={kernel}", flush=True)
        w32 = dict(w)
        for k in ("dtau", "w0", "g0"):
            w32[k] = np.ascontiguousarray(w[k].astype(np.float32).astype(np.float64))
        ref = O.solve(w32, per_bin=True, extended=True)
        s = rt.Solver(w["lambda_edges"], w["F_star"])
        inp = rt.to_device(w, input_f32=True)
        assert inp["dtau"].dtype == torch.float32
        out = s.solve(inp, precision=rt.RT_MIXED, per_bin=True, kernel=kernel)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        got["flags"] = got["flags"].view(np.uint32)
        e = assert_close(got, ref, w["p_iface"], MIXED_TOL, floor=FLOOR[1], floor_bin=FLOOR_BIN[1])
        print(f"  errors={e}", flush=True)
        np.testing.assert_array_equal(got["flags"], ref["flags"])
        with pytest.raises(ValueError):
            s.solve(inp, precision=rt.RT_FP64, kernel=kernel)
        s.close()


def test_strict_mode_flags_edomain(rt, torch):
    w = edge_workload()
    opts = O.Options(e_clamp=0)
    ref = O.solve(w, opts, extended=True)
    out = gpu_solve(rt, torch, w, rt.RT_FP64, opts=opts)
    assert ref["flags"][5] & O.F_EDOMAIN
    np.testing.assert_array_equal(out["flags"], ref["flags"])
    ok = np.array([not (f & O.F_EDOMAIN) for f in ref["flags"]])
    assert_close({k: v[..., ok] if v.ndim == 2 else v for k, v in out.items()
                  if k in ("F_up", "F_dn", "F_beam", "F_net", "heating")},
                 {k: v[..., ok] for k, v in ref.items()
                  if k in ("F_up", "F_dn", "F_beam", "F_net", "heating")},
                 w["p_iface"][:, ok], FP64_TOL)


def test_conservative_scattering_w0_one(rt, torch):
    """w0 = 1 exactly (regular mode), no thermal emission: the oracle's printed
    form is 0/0 there, so the GPU is checked against energy conservation
    (zero net flux at every interface) and against the oracle at w0 = 1 - 1e-15
    (fluxes move by O((1 - w0) tau^2) between the two)."""
    w = small(C=4, N=8, NB=3, seed=41, cloud="none")
    w["w0"] = np.ones_like(w["w0"])
    w["g0"] = np.full_like(w["g0"], 0.4)
    w["T_iface"] = np.full_like(w["T_iface"], 1e-3)     # negligible emission
    w["T_int"] = np.zeros_like(w["T_int"])
    w["mu_star"] = np.array([0.9, 0.6, 0.3, 0.2])
    opts = O.Options(improved=0)
    out = gpu_solve(rt, torch, w, rt.RT_FP64, opts=opts)
    gross = (out["F_up"] + out["F_dn"] + out["F_beam"]).max(axis=0)
    assert np.all(np.abs(out["F_net"]) <= 1e-12 * gross)
    w2 = dict(w)
    w2["w0"] = np.full_like(w["w0"], 1.0 - 1e-15)
    ref = O.solve(w2, opts, extended=True)
    assert_close(out, ref, w["p_iface"], 1e-9, keys=("F_up", "F_dn", "F_beam"))


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_invalid_inputs_flagged(rt, torch, kernel):
    w = small(C=5, N=6, NB=4, seed=51)
    w = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in w.items()}
    w["w0"][2, 1, 0] = 1.5
    w["T_iface"][3, 2] = -5.0
    w["p_iface"][4, 3] = w["p_iface"][3, 3] * 2
    out = gpu_solve(rt, torch, w, rt.RT_FP64, kernel=kernel)
    assert out["flags"][1] & O.F_INVALID and out["flags"][2] & O.F_INVALID
    assert out["flags"][3] & O.F_INVALID
    assert not out["flags"][0] & O.F_INVALID and not out["flags"][4] & O.F_INVALID


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_repeat_is_bitwise_identical(rt, torch, kernel):
    w = small(C=40, N=12, NB=30, seed=61)
    a = gpu_solve(rt, torch, w, rt.RT_FP64, per_bin=True, kernel=kernel)
    b = gpu_solve(rt, torch, w, rt.RT_FP64, per_bin=True, kernel=kernel)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("K", [1, 3, 8, 37])
def test_layer_kernel_tiles(rt, torch, K):
    """Layer kernel with tiles that leave a ragged last workgroup, several
    chunks of levels and a last chunk shorter than the others."""
    w = small(C=37, N=23, NB=7, seed=71)
    print(f"\n[parity] tiles K={K}", flush=True)
    ref = O.solve(w, per_bin=True, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, per_bin=True, kernel=2, cols_per_block=K)
        assert_close(out, ref, w["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec])
        np.testing.assert_array_equal(out["flags"], ref["flags"])


SUB_CASES = [
    ("sub_small", dict(C=7, N=6, NB=5, seed=81)),
    ("sub_bins30", dict(C=23, N=20, NB=30, seed=82)),
    ("sub_one_layer", dict(C=5, N=1, NB=3, seed=83)),
]


@pytest.mark.parametrize("name,shape", SUB_CASES, ids=[c[0] for c in SUB_CASES])
def test_sublayer_grid(rt, torch, name, shape):
    """Sub-layer grid (layers split at their centres): interface and centre
    fluxes, per-bin fluxes at all 2N+1 levels and heating against the oracle."""
    spec = synth.Spec(name="s", g_level=3, n_layers=shape["N"], n_bins=shape["NB"],
                      cloud="night", seed=shape["seed"])
    w = synth.make_sublayer(spec, n_cols=shape["C"])
    print(f"\n[parity] {name} {shape}", flush=True)
    ref = O.solve_sublayer(w, per_bin=True, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, per_bin=True)
        assert "F_net_center" in out and out["F_up_bin"].shape[0] == 2 * shape["N"] + 1
        e = assert_close(out, ref, w["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec])
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"], ref["flags"])


def test_sublayer_cfg1_sampled(rt, torch):
    """GCM size on the sub-layer grid (2562 x 2*40 slabs x 30 bins), 32
    columns checked against the oracle."""
    w = synth.make_sublayer("cfg1")
    cols = np.linspace(0, w["n_cols"] - 1, 32).astype(int)
    ws = subset(w, cols)
    ref = O.solve_sublayer(ws, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec)
        e = assert_close(out, ref, ws["p_iface"], tol, floor=FLOOR[prec],
                         floor_bin=FLOOR_BIN[prec], cols=cols)
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"][cols], ref["flags"])


def test_sublayer_request_errors(rt, torch):
    """The sub-layer grid needs the layer kernel and all four centre outputs."""
    w = synth.make_sublayer(synth.Spec(name="s", g_level=1, n_layers=3, n_bins=2, seed=84),
                            n_cols=2)
    s = rt.Solver(w["lambda_edges"], w["F_star"])
    inp = rt.to_device(w)
    out = s.outputs(2, 3, sublayer=True)
    with pytest.raises(rt.RtError) as e:
        s.solve(inp, out=out, kernel=rt.RT_KERNEL_LANE, cols_per_block=0)
    assert e.value.status == rt.RT_EINVAL
    del out["F_beam_center"]
    with pytest.raises(rt.RtError) as e:
        s.solve(inp, out=out)
    assert e.value.status == rt.RT_EINVAL
    s.close()


KDIST_CASES = [
    ("kd_small", dict(C=5, N=6, NB=4, NG=5, seed=91)),
    ("kd_ragged", dict(C=13, N=9, NB=7, NG=3, seed=92)),
    ("kd_2x20", dict(C=9, N=7, NB=2, NG=20, seed=94)),
]


@pytest.mark.parametrize("name,shape", KDIST_CASES, ids=[c[0] for c in KDIST_CASES])
def test_kdist_bins(rt, torch, name, shape):
    """k-distribution bins (Gaussian points with weights): weighted bin sums,
    per-(bin, g) fluxes and the weighted TOA spectrum against the oracle."""
    spec = synth.Spec(name="k", g_level=3, n_layers=shape["N"], n_bins=shape["NB"],
                      cloud="night", seed=shape["seed"])
    w = synth.make_kdist(spec, n_cols=shape["C"], n_gauss=shape["NG"])
    print(f"\n[parity] {name} {shape}", flush=True)
    ref = O.solve(w, per_bin=True, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, per_bin=True)
        assert out["F_up_bin"].shape[2] == shape["NB"] * shape["NG"]
        e = assert_close(out, ref, w["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec])
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"], ref["flags"])


def test_kdist_paper_shape_sampled(rt, torch):
    """The paper's production spectral set-up: 2562 columns x 40 layers x 30
    bins x 20 Gaussian points (600 solves per column), 16 columns checked."""
    w = synth.make_kdist("cfg1", n_gauss=20)
    cols = np.linspace(0, w["n_cols"] - 1, 16).astype(int)
    ws = subset(w, cols)
    ws["gauss_w"] = w["gauss_w"]
    ref = O.solve(ws, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec)
        e = assert_close(out, ref, ws["p_iface"], tol, floor=FLOOR[prec],
                         floor_bin=FLOOR_BIN[prec], cols=cols)
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"][cols], ref["flags"])


def test_kdist_needs_layer_kernel(rt, torch):
    spec = synth.Spec(name="k", g_level=1, n_layers=3, n_bins=2, seed=93)
    w = synth.make_kdist(spec, n_cols=2, n_gauss=4)
    s = rt.Solver(w["lambda_edges"], w["F_star"], gauss_weights=w["gauss_w"])
    inp = rt.to_device(w)
    with pytest.raises(rt.RtError) as e:
        s.solve(inp, kernel=rt.RT_KERNEL_LANE, cols_per_block=0)
    assert e.value.status == rt.RT_EINVAL
    s.close()


def test_cfg4_sampled(rt, torch):
    """High resolution, 10242 x 80 x 300 with cloud decks up to w0 = 0.9999,
    g0 = 0.98 and dtau log-uniform [1e-8, 1e3]: solved whole on the GPU in
    both precisions, 24 columns checked against the oracle."""
    w = synth.make("cfg4")
    print(f"\n[parity] cfg4 full {w['n_cols']}x{w['n_layers']}x{w['n_bins']}", flush=True)
    cols = np.unique(np.concatenate([np.linspace(0, w["n_cols"] - 1, 16).astype(int),
                                     np.argsort(np.abs(w["mu_star"]))[:8]]))
    ws = subset(w, cols)
    ref = O.solve(ws, extended=True)
    for prec, tol in ((rt.RT_MIXED, MIXED_TOL), (rt.RT_FP64, FP64_TOL)):
        out = gpu_solve(rt, torch, w, prec)
        e = assert_close(out, ref, ws["p_iface"], tol, floor=FLOOR[prec],
                         floor_bin=FLOOR_BIN[prec], cols=cols)
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"][cols], ref["flags"])


def test_request_validation_before_launch(rt, torch):
    """Argument and shape errors of a request reach the C-ABI and return
    RT_EINVAL from rt_solve_fluxes, rt_solve_fluxes_noalloc and rt_submit
    before any launch (the outputs keep their sentinel), and the handle
    solves a valid request afterwards."""
    w = small(C=40, N=6, NB=30, seed=91)
    s = rt.Solver(w["lambda_edges"], w["F_star"])
    inp = rt.to_device(w)
    out = s.outputs(w["n_cols"], w["n_layers"])
    for v in out.values():
        v.fill_(7.0) if v.dtype == torch.float64 else v.fill_(7)
    torch.cuda.synchronize()
    good = s.request(inp, out, rt.RT_FP64, 0, rt.RT_KERNEL_LAYER)
    odd = inp["dtau"].data_ptr() + 4
    broken = {
        "no columns": dict(n_cols=0), "no layers": dict(n_layers=0), "too many layers": dict(n_layers=4097),
        "precision": dict(precision=7), "kernel": dict(kernel=9),
        "deep with a tile": dict(kernel=rt.RT_KERNEL_DEEP, cols_per_block=2),
        "FP32 storage in FP64": dict(input_dtype=1), "negative tile": dict(cols_per_block=-1),
        "lane tile too wide": dict(kernel=rt.RT_KERNEL_LANE, cols_per_block=20), "no dtau": dict(dtau=None),
        "no F_net": dict(F_net=None), "centre without T_center": dict(p_center=inp["p_iface"].data_ptr()),
        "misaligned dtau": dict(dtau=odd),
    }
    for name, change in broken.items():
        req = rt.RtRequest.from_buffer_copy(good)
        for k, v in change.items():
            setattr(req, k, v)
        for call in (lambda r: rt.rt_solve_fluxes(s.h, r, None),
                     lambda r: rt.rt_solve_fluxes_noalloc(s.h, r, None),
                     lambda r: rt.rt_submit(s.h, r)):
            with pytest.raises(rt.RtError) as e:
                call(req)
            assert e.value.status == rt.RT_EINVAL, (name, e.value.status)
    torch.cuda.synchronize()
    assert (out["F_net"] == 7.0).all() and (out["heating"] == 7.0).all()
    ref = s.solve(inp, out=out, kernel=rt.RT_KERNEL_LAYER, cols_per_block=0)
    torch.cuda.synchronize()
    assert torch.isfinite(ref["F_net"]).all()
    s.close()
