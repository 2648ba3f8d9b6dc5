"""A solve captured in a HIP graph (torch.cuda.CUDAGraph around
rt_solve_fluxes_noalloc) replays to the eager result.  The allocation-free entry
point puts only kernel launches on the caller's stream (no allocation, copy or
memset), so its graph replays the same kernels on the same buffers.  Every
replay is checked bit for bit against the eager solve, with the outputs
overwritten by eager work and the device synchronised between replays; layer
and deep kernels (one and seven launches per solve), both precisions."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KEYS = ("F_up", "F_dn", "F_beam", "F_net", "heating", "F_up_toa_bin", "flags")


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def rt(torch):
    from paper_2203_02293_amd import rt as r
    r.lib()
    return r


def host(out):
    return {k: out[k].cpu().numpy() for k in KEYS}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kernel", ["layer", "deep"])
def test_graph_replays_match_eager(rt, torch, precision, kernel):
    from paper_2203_02293_amd import synth
    kid = rt.RT_KERNEL_LAYER if kernel == "layer" else rt.RT_KERNEL_DEEP
    C, N, NB = (162, 40, 30) if kernel == "layer" else (2, 600, 30)
    w = synth.make(synth.Spec(name="graph", g_level=4, n_layers=N, n_bins=NB, cloud="fraction",
                              seed=41), n_cols=C)
    print(f"graph case kernel={kernel} precision={precision} shape={C}x{N}x{NB}", flush=True)
    s = rt.Solver(w["lambda_edges"], w["F_star"])
    inp = rt.to_device(w)
    kw = dict(precision=precision, kernel=kid, cols_per_block=0, noalloc=True)
    ref_out = s.outputs(C, N)
    s.solve(inp, out=ref_out, **kw)
    torch.cuda.synchronize()
    ref = host(ref_out)

    out = s.outputs(C, N)
    side = torch.cuda.Stream()           # warm-up off the default stream, then capture
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        s.solve(inp, out=out, **kw)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.solve(inp, out=out, **kw)
    for rep in range(3):
        for k in KEYS:
            out[k].fill_(7)              # eager work between replays (a fill kernel)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = host(out)
        for k in KEYS:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{k}, replay {rep}")
    del g
    s.close()
