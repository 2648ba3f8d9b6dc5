"""Drive the host builds of the layer kernel (``build.py``) and of the
deep-column kernels (``deep_build.py``) on a workload dict.

Argument structs mirror ``SolveArgs``/``Opts`` of ``csrc/rt_internal.hpp``
field by field.  Test infrastructure only.
"""
import ctypes as ct

import numpy as np

import oracle as O

from . import build as _build

_L = None
dp = ct.c_void_p


def lib():
    global _L
    if _L is None:
        _L = ct.CDLL(str(_build.build()))
    return _L


class Opts(ct.Structure):
    _fields_ = [('improved', ct.c_int), ('noniso', ct.c_int), ('e_clamp', ct.c_int), ('pad_', ct.c_int),
                ('eps2', ct.c_double), ('e_tau', ct.c_double), ('g_guard', ct.c_double),
                ('gravity', ct.c_double), ('cp', ct.c_double)]


class Args(ct.Structure):
    _fields_ = [(n, ct.c_int) for n in ('C', 'N', 'NB', 'K', 'PC', 'CH', 'sub', 'in_f32', 'NG')] + \
        [(n, dp) for n in ('c2', 'c2f', 'F_star', 'wg', 'p', 'T', 'dtau', 'w0', 'g0', 'mu', 'Tint', 'Ftoa',
                           'F_up', 'F_dn', 'F_beam', 'F_net', 'heat', 'dTdt', 'F_up_toa_bin', 'F_up_bin',
                           'F_dn_bin', 'flags', 'status', 'Tc', 'pc', 'F_up_c', 'F_dn_c', 'F_beam_c', 'F_net_c',
                           'scratch')] + [('L', ct.c_longlong), ('o', Opts)]


def geometry(C, NBG, K, mixed, lds=160 * 1024, ncu=256, NG=1, worker=False):
    v = (ct.c_int * 7)()
    lib().emu_geometry(C, NBG, K, int(mixed), lds, ncu, v, NG, int(worker))
    return dict(K=v[0], PC=v[1], CH=v[2], threads=v[3], blocks=v[4], lds=v[5], lanes=v[6])


def solve(w, mixed, K=0, opts=None, lds=160 * 1024, ncu=256, per_bin=True, worker=False):
    """The layer kernel on the host (worker: at the serving worker's tile)."""
    NG = int(w.get('n_gauss', 1)) if w.get('gauss_w') is not None else 1
    g = geometry(w['n_cols'], w['n_bins'] * NG, K, mixed, lds, ncu, NG, worker)
    S = 2 * w['n_layers'] if w.get('T_center') is not None and w.get('sublayer', False) else w['n_layers']
    scratch = np.full(S * 4 * g['lanes'], np.nan)
    out, a, keep = _args(w, opts, per_bin, scratch.ctypes.data)
    lib().emu_solve(ct.byref(a), int(mixed), K, lds, ncu, int(worker))
    return out, g


_DL = None


def deep_lib():
    global _DL
    if _DL is None:
        from . import deep_build
        _DL = ct.CDLL(str(deep_build.build()))
    return _DL


def deep_geometry(C, N, NBG, ncu=256, lds=160 * 1024):
    v = (ct.c_longlong * 8)()
    deep_lib().emu_deep_geometry(C, N, NBG, ncu, lds, v)
    return dict(S=v[0], Ls=v[1], CH=v[2], threads=v[3], blocks=v[4], lds=v[5], lanes=v[6],
                scratch=v[7])


class _Guarded:
    """Host buffer of n bytes (NaN-filled) ending right before an inaccessible
    page: a write or read past its end faults at once."""

    def __init__(self, n):
        import mmap
        libc = ct.CDLL(None, use_errno=True)
        pg = mmap.PAGESIZE
        body = (n + pg - 1) // pg * pg
        self.m = mmap.mmap(-1, body + pg)
        base = ct.addressof(ct.c_char.from_buffer(self.m))
        assert libc.mprotect(ct.c_void_p(base + body), ct.c_size_t(pg), 0) == 0
        ct.memset(base, 0xFF, body)
        self.ptr = base + body - n
        self._base = base


def solve_deep(w, mixed, opts=None, ncu=256, lds=160 * 1024, per_bin=True):
    """The deep-column kernels on the host."""
    NG = int(w.get('n_gauss', 1)) if w.get('gauss_w') is not None else 1
    sub = w.get('T_center') is not None and w.get('sublayer', False)
    S = 2 * w['n_layers'] if sub else w['n_layers']
    g = deep_geometry(w['n_cols'], S, w['n_bins'] * NG, ncu, lds)
    buf = _Guarded(g['scratch'])
    out, a, keep = _args(w, opts, per_bin, buf.ptr)
    rc = deep_lib().emu_deep_solve(ct.byref(a), int(mixed), ncu, lds)
    assert rc == 0
    return out, g


def _args(w, opts, per_bin, scratch_ptr):
    o = opts or O.Options()
    C, N, NB = w['n_cols'], w['n_layers'], w['n_bins']
    NG = int(w.get('n_gauss', 1)) if w.get('gauss_w') is not None else 1
    sub = w.get('T_center') is not None and w.get('sublayer', False)
    S = 2 * N if sub else N
    NBG = NB * NG
    keep = []
    def P(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a)
        keep.append(a)
        return a.ctypes.data
    c2 = 6.62607015e-34 * 299792458.0 / 1.380649e-23 / np.asarray(w['lambda_edges'])
    gw = np.asarray(w['gauss_w']) if NG > 1 else np.ones(1)
    out = {k: np.zeros((N + 1, C)) for k in ('F_up', 'F_dn', 'F_beam', 'F_net')}
    out['heating'] = np.zeros((N, C)); out['dTdt'] = np.zeros((N, C))
    out['F_up_toa_bin'] = np.zeros((C, NB)); out['flags'] = np.zeros(C, dtype=np.uint32)
    out['status'] = np.zeros(1, dtype=np.uint32)
    if per_bin:
        out['F_up_bin'] = np.zeros((S + 1, C, NBG)); out['F_dn_bin'] = np.zeros((S + 1, C, NBG))
    if sub:
        for k in ('F_up_center', 'F_dn_center', 'F_beam_center', 'F_net_center'):
            out[k] = np.zeros((N, C))
    a = Args(C, S, NBG, 0, 0, 0, int(sub), 0, NG, P(c2), P(c2.astype(np.float32)), P(w['F_star']), P(gw),
             P(w['p_iface']), P(w['T_iface']), P(w['dtau']), P(w['w0']), P(w['g0']), P(w['mu_star']),
             P(w['T_int']), P(w.get('F_toa')), out['F_up'].ctypes.data, out['F_dn'].ctypes.data,
             out['F_beam'].ctypes.data, out['F_net'].ctypes.data, out['heating'].ctypes.data,
             out['dTdt'].ctypes.data, out['F_up_toa_bin'].ctypes.data,
             out['F_up_bin'].ctypes.data if per_bin else None,
             out['F_dn_bin'].ctypes.data if per_bin else None, out['flags'].ctypes.data,
             out['status'].ctypes.data, P(w.get('T_center')) if sub else None, P(w.get('p_center')) if sub else None,
             out['F_up_center'].ctypes.data if sub else None, out['F_dn_center'].ctypes.data if sub else None,
             out['F_beam_center'].ctypes.data if sub else None, out['F_net_center'].ctypes.data if sub else None,
             scratch_ptr, 0, Opts(o.improved, o.noniso, o.e_clamp, 0, o.eps2, o.e_tau, o.g_guard,
                                  o.gravity, o.cp))
    return out, a, keep
