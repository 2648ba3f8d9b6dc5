"""rt_solve_fluxes_noalloc: the allocation-free variant of rt_solve_fluxes
gives the same results as rt_solve_fluxes on the same requests, on two calls
in a row (the second smaller, so the shared static work buffer holds the
first call's data), for the layer and deep kernels, both precisions; and a
request whose work buffer exceeds the static array is refused before any
launch."""
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
    return r


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def work(synth, C, N, NB, seed):
    return synth.make(synth.Spec(name="noalloc", g_level=4, n_layers=N, n_bins=NB,
                                 cloud="night", seed=seed), n_cols=C)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kernel", ["layer", "deep"])
def test_noalloc_matches_solve(rt, torch, precision, kernel):
    from paper_2203_02293_amd import synth
    kid = rt.RT_KERNEL_LAYER if kernel == "layer" else rt.RT_KERNEL_DEEP
    shapes = [(162, 40, 30), (37, 17, 30)] if kernel == "layer" else [(2, 600, 30), (1, 300, 30)]
    w0 = work(synth, *shapes[0], seed=21)
    s = rt.Solver(w0["lambda_edges"], w0["F_star"])
    for i, (C, N, NB) in enumerate(shapes):
        w = work(synth, C, N, NB, seed=21 + i)
        inp = rt.to_device(w)
        print(f"noalloc case kernel={kernel} precision={precision} shape={C}x{N}x{NB}", flush=True)
        ref = s.solve(inp, precision=precision, kernel=kid, cols_per_block=0)
        out = s.outputs(C, N)
        torch.cuda.synchronize()
        got = s.solve(inp, precision=precision, kernel=kid, cols_per_block=0, out=out,
                      noalloc=True)
        torch.cuda.synchronize()
        r, g = host(ref), host(got)
        for k in ("F_up", "F_dn", "F_beam", "F_net", "heating", "F_up_toa_bin", "flags"):
            np.testing.assert_array_equal(g[k], r[k], err_msg=f"{k} at {C}x{N}x{NB}")
    s.close()


def test_noalloc_refuses_oversized_request(rt, torch):
    from paper_2203_02293_amd import synth
    w = work(synth, 2562, 120, 30, seed=5)     # FP64 work buffer of ~300 MB
    s = rt.Solver(w["lambda_edges"], w["F_star"])
    assert s.work_bytes(w["n_cols"], w["n_layers"]) > 128 << 20
    inp = rt.to_device(w)
    out = s.outputs(w["n_cols"], w["n_layers"])
    with pytest.raises(rt.RtError) as e:
        s.solve(inp, kernel=rt.RT_KERNEL_LAYER, cols_per_block=0, out=out, noalloc=True)
    assert e.value.status == rt.RT_ENOMEM
    s.close()
