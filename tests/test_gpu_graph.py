"""A solve captured in a HIP graph (torch.cuda.CUDAGraph around
rt_solve_fluxes_noalloc) replays to the eager result.  The allocation-free entry
point puts only kernel launches on the caller's stream (no allocation, copy or
memset), so its graph replays the same kernels on the same buffers.  Every
replay is checked bit for bit against the eager solve, with the outputs
overwritten by eager work and the device synchronised between replays, in both
precisions: the layer kernel with wavefront bin sums, the deep kernel (seven
launches), k-distribution bins (the layer kernel's LDS-staged
back-substitution), the sub-layer grid (centre outputs as well), and on the
mixed path FP32 storage of the layer inputs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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
    return {k: v.cpu().numpy() for k, v in out.items()}


def workload(synth, kind):
    """A small request of each kind (host arrays) and the kernel it runs on."""
    if kind == "layer":
        spec = synth.Spec(name="graph", g_level=4, n_layers=40, n_bins=30, cloud="fraction", seed=41)
        return synth.make(spec, n_cols=162), "layer"
    if kind == "deep":
        spec = synth.Spec(name="graph", g_level=4, n_layers=600, n_bins=30, cloud="fraction", seed=42)
        return synth.make(spec, n_cols=2), "deep"
    if kind == "kdist":
        spec = synth.Spec(name="graph", g_level=3, n_layers=20, n_bins=10, cloud="night", seed=43)
        return synth.make_kdist(spec, n_cols=40, n_gauss=12), "layer"
    spec = synth.Spec(name="graph", g_level=3, n_layers=12, n_bins=30, cloud="night", seed=44)
    return synth.make_sublayer(spec, n_cols=50), "layer"


# (kind, precision); in32: the layer request with dtau, w0, g0 stored as floats
# (mixed path only)
CASES = [(k, p) for k in ("layer", "deep", "kdist", "sublayer") for p in (0, 1)] + [("in32", 1)]


@pytest.mark.parametrize("kind,precision", CASES, ids=[f"{k}-{p}" for k, p in CASES])
def test_graph_replays_match_eager(rt, torch, kind, precision):
    from paper_2203_02293_amd import synth
    w, kname = workload(synth, "layer" if kind == "in32" else kind)
    kid = rt.RT_KERNEL_LAYER if kname == "layer" else rt.RT_KERNEL_DEEP
    C, N = w["n_cols"], w["n_layers"]
    sub = kind == "sublayer"
    print(f"graph case {kind} precision={precision} shape={C}x{N}x{w['n_bins']}", flush=True)
    s = rt.Solver(w["lambda_edges"], w["F_star"], gauss_weights=w.get("gauss_w"))
    inp = rt.to_device(w, input_f32=kind == "in32")
    kw = dict(precision=precision, kernel=kid, cols_per_block=0, noalloc=True)
    ref_out = s.outputs(C, N, sublayer=sub)
    s.solve(inp, out=ref_out, **kw)
    torch.cuda.synchronize()
    ref = host(ref_out)

    out = s.outputs(C, N, sublayer=sub)
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
        for v in out.values():
            v.fill_(7)                   # eager work between replays (a fill kernel)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = host(out)
        for k in ref:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{k}, replay {rep}")
    del g
    s.close()
