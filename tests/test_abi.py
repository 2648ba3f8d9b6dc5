"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
public header declares, and its host-side argument checks reject bad
configurations before touching a device (no compute calls here)."""
import ctypes as ct
import pathlib
import re

import numpy as np
import pytest

from paper_2203_02293_amd import rt

ROOT = pathlib.Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "rt.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2203_02293_amd import build
    if build.stale():
        build.build()
    return rt.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert set(names) == set(rt.SYMBOLS)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for s in (rt.RT_OK, rt.RT_PENDING, rt.RT_EINVAL, rt.RT_ENOMEM, rt.RT_EDEVICE,
              rt.RT_EDOMAIN, rt.RT_EBUSY, rt.RT_ENOTFOUND):
        assert lib.rt_status_string(s)
    assert lib.rt_status_string(12345) == b"unknown status"


def test_config_defaults_follow_table3(lib):
    c = rt.rt_config_default()
    assert (c.improved, c.noniso, c.e_clamp) == (1, 1, 1)
    assert c.eps2 == pytest.approx(2 / 3) and c.e_tau == 1e-4 and c.g_guard == 1e-5
    assert c.gravity == 47.0 and c.cp == 12436.0


def _cfg(nb=3, lam=None, fs=None):
    c = rt.rt_config_default()
    lam = np.array([1e-6, 2e-6, 3e-6, 4e-6]) if lam is None else lam
    fs = np.ones(nb) if fs is None else fs
    c.n_bins = nb
    c.lambda_edges = lam.ctypes.data_as(ct.POINTER(ct.c_double))
    c.stellar_flux = fs.ctypes.data_as(ct.POINTER(ct.c_double))
    return c, lam, fs


@pytest.mark.parametrize("mutate", [
    lambda c: setattr(c, "n_bins", 0),
    lambda c: setattr(c, "n_bins", 513),
    lambda c: setattr(c, "eps2", 0.0),
    lambda c: setattr(c, "gravity", -1.0),
    lambda c: setattr(c, "e_tau", -1.0),
    lambda c: setattr(c, "max_inflight", -2),
])
def test_create_rejects_bad_config(lib, mutate):
    c, lam, fs = _cfg()
    mutate(c)
    h = ct.c_void_p()
    assert lib.rt_create(ct.byref(c), ct.byref(h)) == rt.RT_EINVAL
    assert h.value is None


def test_create_rejects_unsorted_edges_and_negative_flux(lib):
    c, lam, fs = _cfg(lam=np.array([1e-6, 3e-6, 2e-6, 4e-6]))
    h = ct.c_void_p()
    assert lib.rt_create(ct.byref(c), ct.byref(h)) == rt.RT_EINVAL
    c, lam, fs = _cfg(fs=np.array([1.0, -1.0, 1.0]))
    assert lib.rt_create(ct.byref(c), ct.byref(h)) == rt.RT_EINVAL


def test_null_arguments(lib):
    h = ct.c_void_p()
    assert lib.rt_create(None, ct.byref(h)) == rt.RT_EINVAL
    assert lib.rt_destroy(None) == rt.RT_OK
    assert lib.rt_solve_fluxes(None, None, None) == rt.RT_EINVAL
    assert lib.rt_request_kernel(None, None) == rt.RT_EINVAL
    assert lib.rt_poll(None, 1) == rt.RT_EINVAL
    assert lib.rt_last_error(None) == b"null handle"
