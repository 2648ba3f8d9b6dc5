"""CPU checks of the Python binding's host logic: request tensors are checked
against the layouts of include/rt.h before anything reaches the library, and
the autotuner's table is only applied to the requests it was measured on."""
import numpy as np
import pytest
import torch

from paper_2203_02293_amd import rt, synth


def host_request(C=5, N=4, NB=3, sub=False):
    if sub:
        w = synth.make_sublayer(synth.Spec(name="t", g_level=1, n_layers=N, n_bins=NB, seed=1),
                                n_cols=C)
        keys = ("p_iface", "T_iface", "dtau", "w0", "g0", "mu_star", "T_int", "T_center",
                "p_center")
    else:
        w = synth.make(synth.Spec(name="t", g_level=1, n_layers=N, n_bins=NB, seed=1), n_cols=C)
        keys = ("p_iface", "T_iface", "dtau", "w0", "g0", "mu_star", "T_int")
    inp = {k: torch.from_numpy(np.ascontiguousarray(w[k])) for k in keys}
    f = dict(dtype=torch.float64)
    out = {k: torch.empty((N + 1, C), **f) for k in ("F_up", "F_dn", "F_beam", "F_net")}
    out["heating"] = torch.empty((N, C), **f)
    out["flags"] = torch.zeros(C, dtype=torch.int32)
    if sub:
        for k in ("F_up_center", "F_dn_center", "F_beam_center", "F_net_center"):
            out[k] = torch.empty((N, C), **f)
    return inp, out


def rejects(inp, out, msg, C=5, N=4, NB=3, NG=1, sub=False, precision=rt.RT_FP64):
    with pytest.raises(ValueError, match=msg):
        rt.check_request(inp, out, C, N, NB, NG, sub, precision)


def test_float32_inputs_rejected():
    """A float32 optical-depth tensor (torch's default dtype) would be read as
    doubles past its end: refused before any launch."""
    inp, out = host_request()
    for k in ("dtau", "w0", "g0", "p_iface", "mu_star"):
        bad = dict(inp, **{k: inp[k].float()})
        rejects(bad, out, f"{k} must be float64")


def test_float32_storage_of_layer_inputs():
    """dtau, w0 and g0 all float32 is the mixed path's FP32 input storage
    (RT_F32): accepted with RT_MIXED (the host request then stops only at the
    device check), refused with RT_FP64; one of them alone stays an error."""
    inp, out = host_request()
    f32 = dict(inp, **{k: inp[k].float() for k in ("dtau", "w0", "g0")})
    rejects(f32, out, "need the mixed precision")
    rejects(f32, out, "contiguous device tensor", precision=rt.RT_MIXED)
    rejects(dict(f32, p_iface=inp["p_iface"].float()), out, "p_iface must be float64",
            precision=rt.RT_MIXED)
    rejects(dict(inp, w0=inp["w0"].float()), out, "w0 must be float64", precision=rt.RT_MIXED)


def test_short_or_misshaped_tensors_rejected():
    inp, out = host_request()
    rejects(dict(inp, dtau=inp["dtau"][:, :4]), out, "dtau must have shape")
    rejects(inp, dict(out, F_up=out["F_up"][:4]), "F_up must have shape")
    rejects(inp, dict(out, heating=torch.empty((5, 5), dtype=torch.float64)),
            "heating must have shape")
    rejects(inp, dict(out, flags=torch.zeros(5, dtype=torch.float64)), "flags must be int32")
    rejects(inp, dict(out, F_up_bin=torch.empty((5, 5, 2), dtype=torch.float64)),
            "F_up_bin must have shape")
    # with Gaussian points per bin every per-lane array has NB x NG entries
    rejects(inp, out, "dtau must have shape", NG=4)


def test_sublayer_shapes():
    inp, out = host_request(sub=True)
    # 2N slabs and 2N+1 levels of per-bin fluxes on the sub-layer grid
    rejects(inp, dict(out, F_up_bin=torch.empty((5, 5, 3), dtype=torch.float64)),
            "F_up_bin must have shape", sub=True)
    rejects(dict(inp, p_center=None), out, "p_center is required", sub=True)
    # a well-formed host request passes every shape and dtype check and stops
    # only at the device check
    rejects(inp, out, "contiguous device tensor", sub=True)


def test_tuned_launch_plain_requests_only():
    """The table's entries are plain requests (one slab per layer, one point
    per bin); a sub-layer or k-distribution request with the same lane count
    gets the library defaults (a kernel that runs it), never a lane-kernel
    entry."""
    kern, K = rt.tuned_launch(100, rt.RT_MIXED, 2562, 40)
    assert (kern, K) != (0, 0)
    assert rt.tuned_launch(100, rt.RT_MIXED, 2562, 40, sublayer=True) == (0, 0)
    assert rt.tuned_launch(100, rt.RT_MIXED, 2562, 40, n_gauss=20) == (0, 0)
    assert rt.tuned_launch(30, rt.RT_FP64, 1, 40)[1] <= 1
