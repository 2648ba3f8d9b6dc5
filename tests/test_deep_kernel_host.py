"""The deep-column kernels (``csrc/rt_deep.hip``) run on the CPU through their
host build (``tests/host_emu/deep_build.py``: one OS thread per GPU thread,
the library's own launch sequence, the work buffer and LDS each ending at an
inaccessible page) against the oracle.  The compute-unit count is varied to
move the segment split: one segment, ragged last segments, scan groups of 1
to 256 threads.  Host arithmetic differs from the device's in the reciprocal
only, so the GPU parity bars apply."""
import numpy as np
import pytest

import oracle as O
from paper_2203_02293_amd import synth
from tests.parity import FLOOR, FLOOR_BIN, errors

run = pytest.importorskip("tests.host_emu.run")


def work(C, N, NB, seed, cloud="night", mu=None, **kw):
    spec = synth.Spec(name="d", g_level=3, n_layers=N, n_bins=NB, cloud=cloud, seed=seed, **kw)
    if mu is None:
        mu = np.linspace(-0.4, 0.95, C) if C > 1 else np.array([0.6])
    return synth.make(spec, n_cols=C, mu_star=mu)


def check(w, mixed, ncu, opts=None):
    sub = w.get("sublayer", False)
    ref = (O.solve_sublayer if sub else O.solve)(w, opts, per_bin=True, extended=True)
    out, g = run.solve_deep(w, mixed, opts=opts, ncu=ncu)
    tol = 1e-5 if mixed else 1e-10
    e = errors(out, ref, w["p_iface"], floor=FLOOR[int(mixed)],
               floor_bin=FLOOR_BIN[int(mixed)])
    bad = {k: v for k, v in e.items() if not v <= tol}
    assert not bad, (g, bad)
    np.testing.assert_array_equal(out["flags"], ref["flags"])
    return g


# (C, N, NB, seed, compute units) -> segments
CASES = [("segments38", (1, 300, 6, 21, 256)),     # 38 segments of 8, scan groups of 64
         ("ragged_tail", (3, 77, 7, 22, 16)),      # 10 segments, the last of 5 slabs
         ("one_segment", (5, 20, 4, 23, 2)),
         ("one_layer", (2, 1, 5, 24, 256)),
         ("bins70", (1, 40, 70, 25, 64)),          # two wavefronts per lane group
         ("one_bin", (4, 50, 1, 26, 64)),
         ("scan256", (1, 1100, 3, 27, 256))]       # 138 segments: scan groups of 256


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name,shape", CASES, ids=[c[0] for c in CASES])
def test_shapes(name, shape, mixed):
    C, N, NB, seed, ncu = shape
    g = check(work(C, N, NB, seed), mixed, ncu)
    assert g["S"] * g["Ls"] >= N and (g["S"] - 1) * g["Ls"] < N


def test_segment_split():
    """Segments of at least 8 slabs, about two workgroups per compute unit."""
    g = run.deep_geometry(1, 4096, 30, 256)
    assert (g["S"], g["Ls"]) == (256, 16)
    g = run.deep_geometry(16, 1000, 30, 256)
    assert (g["S"], g["Ls"]) == (32, 32)
    g = run.deep_geometry(2562, 40, 30, 256)
    assert (g["S"], g["Ls"]) == (1, 40)


def test_thick_scattering_clouds():
    """Dayside cloud decks of w0 up to 0.9999 and optical depths to 1e3:
    c near 1 and eps near 0 across segment boundaries."""
    w = work(4, 200, 8, 31, cloud="fraction", cloud_fraction=1.0, dtau_hi=1e3,
             cloud_w0_hi=0.9999, cloud_g0_hi=0.98, cloud_p_hi_bar=10.0)
    for mixed in (False, True):
        check(w, mixed, 32)


def test_sublayer_grid():
    w = synth.make_sublayer(synth.Spec(name="s", g_level=3, n_layers=30, n_bins=5, cloud="night",
                                       seed=81), n_cols=3)
    for mixed in (False, True):
        check(w, mixed, 16)


def test_kdist_bins():
    w = synth.make_kdist(synth.Spec(name="k", g_level=3, n_layers=40, n_bins=5, cloud="night",
                                    seed=92), n_cols=2, n_gauss=3)
    for mixed in (False, True):
        check(w, mixed, 32)


def test_most_lanes_per_column():
    """256 bins x 3 Gaussian points = 768 lanes, the most a column may hold:
    the per-lane kernels at their workgroup bound, one item per pass."""
    w = synth.make_kdist(synth.Spec(name="k", g_level=3, n_layers=9, n_bins=256, cloud="night",
                                    seed=93), n_cols=1, n_gauss=3)
    g = check(w, False, 256)
    assert g["threads"] == 768


def test_modes_and_edges():
    from tests.test_gpu_parity import edge_workload
    w = edge_workload()
    for opts in (O.Options(), O.Options(improved=0), O.Options(noniso=0)):
        check(w, False, 64, opts=opts)
