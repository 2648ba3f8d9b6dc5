"""GPU parity of the optical-properties step (k-table interpolation, Rayleigh
scattering, gas/condensate mixing; one slab per layer and the sub-layer grid)
against the oracle, element by element, and of optics followed by the solve."""
import numpy as np
import pytest

import oracle as O
from paper_2203_02293_amd import synth
from tests.parity import FLOOR, FLOOR_BIN, TOL, assert_close

pytestmark = pytest.mark.gpu

OPTICS_REL = 1e-12   # dtau: same formulas, rounding only
OPTICS_ABS = 1e-13   # w0, g0 in [0, 1]


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


def setup(rt, C, N, NB, NG, seed):
    spec = synth.Spec(name="o", g_level=4, n_layers=N, n_bins=NB, cloud="night", seed=seed)
    atm = synth.make_atmosphere(spec, n_cols=C)
    tab = synth.opacity_table(NB, NG, seed=seed + 1)
    gw = synth.gauss_points(NG)[1] if NG > 1 else None
    s = rt.Solver(atm["lambda_edges"], atm["F_star"], gauss_weights=gw)
    s.set_opacities(tab)
    return atm, tab, gw, s


def device_atm(torch, atm):
    return {k: torch.from_numpy(np.ascontiguousarray(atm[k])).cuda()
            for k in ("p_iface", "T_iface", "p_center", "T_center")}


# lanes per column (bins x points): within one wavefront pass (6, 24), three
# passes with a ragged last (143), and the paper-like 30 x 20 (ten passes)
@pytest.mark.parametrize("NB,NG", [(6, 1), (6, 4), (13, 11), (30, 20)])
@pytest.mark.parametrize("sublayer", [False, True])
def test_optics_elementwise(rt, torch, NB, NG, sublayer):
    atm, tab, gw, s = setup(rt, C=37, N=11, NB=NB, NG=NG, seed=300 + NG)
    print(f"\n[optics] NB={NB} NG={NG} sublayer={sublayer}", flush=True)
    out = s.optical_properties(device_atm(torch, atm), sublayer=sublayer)
    torch.cuda.synchronize()
    ref = O.optics(atm, tab, sublayer=sublayer)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    err = np.max(np.abs(g["dtau"] - ref["dtau"]) / np.maximum(ref["dtau"], 1e-300))
    assert err <= OPTICS_REL, err
    for k in ("w0", "g0"):
        e = np.max(np.abs(g[k] - ref[k]))
        assert e <= OPTICS_ABS, (k, e)
    s.close()


def test_optics_then_solve(rt, torch):
    """The paper's production pipeline shape in small: k-table bins with
    Gaussian points on the sub-layer grid, optics then fluxes, against the
    oracle's optics then fluxes."""
    atm, tab, gw, s = setup(rt, C=9, N=8, NB=5, NG=4, seed=310)
    dev = device_atm(torch, atm)
    opt = s.optical_properties(dev, sublayer=True)
    inp = dict(dev, **opt, mu_star=torch.from_numpy(atm["mu_star"]).cuda(),
               T_int=torch.from_numpy(atm["T_int"]).cuda())
    ropt = O.optics(atm, tab, sublayer=True)
    ref = O.solve_sublayer(dict(atm, gauss_w=gw, **ropt), per_bin=True, extended=True)
    for prec in (rt.RT_FP64, rt.RT_MIXED):
        tol, floor, fbin = TOL[prec], FLOOR[prec], FLOOR_BIN[prec]
        out = s.solve(inp, precision=prec, per_bin=True)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items()}
        res["flags"] = res["flags"].view(np.uint32)
        e = assert_close(res, ref, atm["p_iface"], tol, floor=floor, floor_bin=fbin)
        print(f"  precision={prec} errors={e}", flush=True)
        np.testing.assert_array_equal(res["flags"], ref["flags"])
    s.close()


def test_optics_errors(rt, torch):
    spec = synth.Spec(name="o", g_level=1, n_layers=3, n_bins=2, seed=5)
    atm = synth.make_atmosphere(spec, n_cols=2)
    s = rt.Solver(atm["lambda_edges"], atm["F_star"])
    with pytest.raises(rt.RtError) as e:
        s.optical_properties(device_atm(torch, atm))
    assert e.value.status == rt.RT_EINVAL
    tab = synth.opacity_table(2, 1)
    bad = dict(tab, temp=tab["temp"][::-1].copy())
    with pytest.raises(rt.RtError) as e:
        s.set_opacities(bad)
    assert e.value.status == rt.RT_EINVAL
    wrong = dict(tab, kappa=np.ones((28, 60, 3)))   # 3 != NB * NG
    with pytest.raises((rt.RtError, ValueError, IndexError)):
        s.set_opacities(wrong)
    s.close()
