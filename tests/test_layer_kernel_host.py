"""The layer kernel's workgroup code run on the CPU (one OS thread per GPU
thread, std::barrier for the workgroup barrier; ``tests/host_emu``) against
the oracle: every phase, index and barrier of the kernel is exercised without
a GPU.  Host arithmetic differs from the device's in the reciprocal only, so
the GPU parity bars apply."""
import numpy as np
import pytest

import oracle as O
from paper_2203_02293_amd import synth
from tests.parity import FLOOR, FLOOR_BIN, errors

run = pytest.importorskip("tests.host_emu.run")


def small(C, N, NB, seed, cloud="night"):
    return synth.make(synth.Spec(name="t", g_level=3, n_layers=N, n_bins=NB, cloud=cloud,
                                 seed=seed), n_cols=C)


def check(w, mixed, K=0, opts=None):
    sub = w.get("sublayer", False)
    ref = (O.solve_sublayer if sub else O.solve)(w, opts, per_bin=True, extended=True)
    out, g = run.solve(w, mixed, K, opts)
    tol = 1e-5 if mixed else 1e-10
    e = errors(out, ref, w["p_iface"], floor=FLOOR[int(mixed)],
               floor_bin=FLOOR_BIN[int(mixed)])
    bad = {k: v for k, v in e.items() if not v <= tol}
    assert not bad, (g, bad)
    np.testing.assert_array_equal(out["flags"], ref["flags"])
    return g


CASES = [("ragged", (37, 9, 7, 11)), ("bins30", (19, 17, 30, 12)), ("one_col", (1, 5, 3, 13)),
         ("one_bin", (300, 4, 1, 14)), ("one_layer", (9, 1, 5, 15)), ("deep", (4, 120, 10, 17)),
         ("bins8", (21, 7, 8, 18)), ("bins40", (13, 9, 40, 19))]


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name,shape", CASES, ids=[c[0] for c in CASES])
def test_shapes(name, shape, mixed):
    check(small(*shape), mixed)


@pytest.mark.parametrize("K", [3, 8, 37])
def test_tiles(K):
    g = check(small(37, 23, 7, 71), False, K=K)
    assert g["K"] == K


def test_gcm_tile_shape():
    """The tile the library picks at 2562 x 40 x 30 (11 columns, several chunks
    per workgroup), on 22 of its columns."""
    from tests.parity import subset
    w = subset(synth.make("cfg1"), np.arange(0, 2562, 116)[:22])
    for mixed in (False, True):
        g = check(w, mixed, K=11)
        assert g["K"] == 11 and g["blocks"] == 2


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
def test_sublayer_grid(mixed):
    w = synth.make_sublayer(synth.Spec(name="s", g_level=3, n_layers=6, n_bins=5, cloud="night",
                                       seed=81), n_cols=7)
    check(w, mixed)


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
@pytest.mark.parametrize("nb,ng", [(7, 3), (2, 20)], ids=["7x3", "2x20"])
def test_kdist_bins(mixed, nb, ng):
    w = synth.make_kdist(synth.Spec(name="k", g_level=3, n_layers=9, n_bins=nb, cloud="night",
                                    seed=92), n_cols=13, n_gauss=ng)
    check(w, mixed)


def test_modes_and_edges():
    from tests.test_gpu_parity import edge_workload
    w = edge_workload()
    for opts in (O.Options(), O.Options(improved=0), O.Options(noniso=0)):
        check(w, False, opts=opts)
    check(w, True)


def test_status_word():
    """The request's status word carries the condition bits that fail a served
    request: F_INVALID from out-of-domain inputs, F_EDOMAIN in strict mode;
    nothing for a clean request or for benign flags (e_tau, clamp)."""
    w = small(9, 6, 5, 52)
    out, _ = run.solve(w, False)
    assert out["status"][0] == 0 and out["flags"].any()     # e_tau flags are benign
    bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in w.items()}
    bad["w0"][2, 3, 1] = 1.5
    out, _ = run.solve(bad, True)
    assert out["status"][0] == O.F_INVALID and out["flags"][3] & O.F_INVALID
    cloud = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in w.items()}
    cloud["w0"][:, 4, :] = 0.999
    cloud["g0"][:, 4, :] = 0.95
    out, _ = run.solve(cloud, False, opts=O.Options(e_clamp=0))
    assert out["status"][0] == O.F_EDOMAIN
    out, _ = run.solve(cloud, False)
    assert out["status"][0] == 0 and out["flags"][4] & O.F_ECLAMP
