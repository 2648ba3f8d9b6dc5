"""GPU parity of the deep-column kernel (RT_KERNEL_DEEP) at the shapes it is
for: few columns of hundreds to thousands of layers, split into segments
over the chip.  Same bars as ``test_gpu_parity.py``: FP64 <= 1e-10, mixed
<= 1e-5 against the oracle's extended-precision build, flags exact."""
import numpy as np
import pytest

import oracle as O
from paper_2203_02293_amd import synth
from tests.parity import assert_close
from tests.test_gpu_parity import (FLOOR, FLOOR_BIN, FP64_TOL, MIXED_TOL, gpu_solve, rt,  # noqa: F401
                                   torch)

pytestmark = pytest.mark.gpu

DEEP = 3   # RT_KERNEL_DEEP


def deep_work(C, N, NB, seed, **kw):
    spec = synth.Spec(name="deep", g_level=3, n_layers=N, n_bins=NB, seed=seed, **kw)
    mu = np.linspace(-0.3, 0.9, C) if C > 1 else np.array([0.5])
    return synth.make(spec, n_cols=C, mu_star=mu)


SHAPES = [("c1_n4096", (1, 4096, 30)), ("c4_n1024", (4, 1024, 30)), ("c16_n512", (16, 512, 30)),
          ("c64_n256", (64, 256, 30)), ("c3_n777_ragged", (3, 777, 7))]


@pytest.mark.parametrize("name,shape", SHAPES, ids=[s[0] for s in SHAPES])
def test_deep_columns(rt, torch, name, shape):
    C, N, NB = shape
    print(f"\n[deep] {name} {shape}", flush=True)
    w = deep_work(C, N, NB, seed=500 + C, cloud="fraction", cloud_fraction=0.5)
    ref = O.solve(w, per_bin=True, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, per_bin=True, kernel=DEEP)
        e = assert_close(out, ref, w["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec])
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"], ref["flags"])


def test_deep_thick_clouds(rt, torch):
    """Dayside decks of w0 to 0.9999 and optical depths to 1e3 over 1000
    layers: c near 1 and eps near 0 at the segment boundaries."""
    w = deep_work(4, 1000, 30, seed=541, cloud="fraction", cloud_fraction=1.0, dtau_hi=1e3,
                  cloud_w0_hi=0.9999, cloud_g0_hi=0.98, cloud_p_hi_bar=10.0)
    ref = O.solve(w, per_bin=True, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, per_bin=True, kernel=DEEP)
        e = assert_close(out, ref, w["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec])
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"], ref["flags"])


def test_deep_sublayer_grid(rt, torch):
    w = synth.make_sublayer(synth.Spec(name="s", g_level=3, n_layers=600, n_bins=30, cloud="night",
                                       seed=551), n_cols=2)
    ref = O.solve_sublayer(w, per_bin=True, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, per_bin=True, kernel=DEEP)
        e = assert_close(out, ref, w["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec])
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"], ref["flags"])


def test_deep_kdist_bins(rt, torch):
    w = synth.make_kdist(synth.Spec(name="k", g_level=3, n_layers=300, n_bins=30, cloud="night",
                                    seed=561), n_cols=2, n_gauss=20)
    ref = O.solve(w, per_bin=True, extended=True)
    for prec, tol in ((rt.RT_FP64, FP64_TOL), (rt.RT_MIXED, MIXED_TOL)):
        out = gpu_solve(rt, torch, w, prec, per_bin=True, kernel=DEEP)
        e = assert_close(out, ref, w["p_iface"], tol, floor=FLOOR[prec], floor_bin=FLOOR_BIN[prec])
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(out["flags"], ref["flags"])


def test_auto_choice(rt, torch):
    """AUTO runs the deep kernel for one column of 4096 layers and the layer
    kernel at GCM size: bitwise the explicit kernel's output in both cases."""
    w = deep_work(1, 4096, 30, seed=571)
    for prec in (rt.RT_FP64, rt.RT_MIXED):
        a = gpu_solve(rt, torch, w, prec)
        d = gpu_solve(rt, torch, w, prec, kernel=DEEP)
        for k in a:
            np.testing.assert_array_equal(a[k], d[k])
    w = synth.make("cfg0")
    a = gpu_solve(rt, torch, w, rt.RT_FP64)
    lay = gpu_solve(rt, torch, w, rt.RT_FP64, kernel=rt.RT_KERNEL_LAYER)
    for k in a:
        np.testing.assert_array_equal(a[k], lay[k])


def test_deep_request_errors(rt, torch):
    w = deep_work(2, 300, 30, seed=581)
    s = rt.Solver(w["lambda_edges"], w["F_star"])
    inp = rt.to_device(w)
    out = s.outputs(2, 300)
    with pytest.raises(rt.RtError, match="cols_per_block"):
        s.solve(inp, out=out, kernel=DEEP, cols_per_block=2)
    with pytest.raises(rt.RtError, match="cols_per_block"):
        s.submit(inp, out, kernel=DEEP, cols_per_block=2)
    assert s.kernel_for(inp, out) == DEEP
    assert s.kernel_for(inp, out, kernel=rt.RT_KERNEL_LAYER) == rt.RT_KERNEL_LAYER
    s.close()
