"""Drive the host build of the layer kernel (``build.py``) on a workload dict.

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
    _fields_ = [(n, ct.c_int) for n in ('C', 'N', 'NB', 'K', 'PC', 'CH', 'sub', 'NG')] + \
        [(n, dp) for n in ('c2', 'c2f', 'F_star', 'wg', 'p', 'T', 'dtau', 'w0', 'g0', 'mu', 'Tint', 'Ftoa',
                           'F_up', 'F_dn', 'F_beam', 'F_net', 'heat', 'dTdt', 'F_up_toa_bin', 'F_up_bin',
                           'F_dn_bin', 'flags', 'Tc', 'pc', 'F_up_c', 'F_dn_c', 'F_beam_c', 'F_net_c',
                           'scratch')] + [('L', ct.c_longlong), ('o', Opts)]


def geometry(C, NBG, K, mixed, lds=160 * 1024, ncu=256):
    v = (ct.c_int * 7)()
    lib().emu_geometry(C, NBG, K, int(mixed), lds, ncu, v)
    return dict(K=v[0], PC=v[1], CH=v[2], threads=v[3], blocks=v[4], lds=v[5], lanes=v[6])


def solve(w, mixed, K=0, opts=None, lds=160 * 1024, ncu=256, per_bin=True):
    o = opts or O.Options()
    C, N, NB = w['n_cols'], w['n_layers'], w['n_bins']
    NG = int(w.get('n_gauss', 1)) if w.get('gauss_w') is not None else 1
    sub = w.get('T_center') is not None and w.get('sublayer', False)
    S = 2 * N if sub else N
    NBG = NB * NG
    g = geometry(C, NBG, K, mixed, lds, ncu)
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
    if per_bin:
        out['F_up_bin'] = np.zeros((S + 1, C, NBG)); out['F_dn_bin'] = np.zeros((S + 1, C, NBG))
    if sub:
        for k in ('F_up_center', 'F_dn_center', 'F_beam_center', 'F_net_center'):
            out[k] = np.zeros((N, C))
    scratch = np.full(S * 4 * g['lanes'], np.nan)
    a = Args(C, S, NBG, 0, 0, 0, int(sub), NG, P(c2), P(c2.astype(np.float32)), P(w['F_star']), P(gw),
             P(w['p_iface']), P(w['T_iface']), P(w['dtau']), P(w['w0']), P(w['g0']), P(w['mu_star']),
             P(w['T_int']), P(w.get('F_toa')), out['F_up'].ctypes.data, out['F_dn'].ctypes.data,
             out['F_beam'].ctypes.data, out['F_net'].ctypes.data, out['heating'].ctypes.data,
             out['dTdt'].ctypes.data, out['F_up_toa_bin'].ctypes.data,
             out['F_up_bin'].ctypes.data if per_bin else None,
             out['F_dn_bin'].ctypes.data if per_bin else None, out['flags'].ctypes.data,
             P(w.get('T_center')) if sub else None, P(w.get('p_center')) if sub else None,
             out['F_up_center'].ctypes.data if sub else None, out['F_dn_center'].ctypes.data if sub else None,
             out['F_beam_center'].ctypes.data if sub else None, out['F_net_center'].ctypes.data if sub else None,
             scratch.ctypes.data, 0, Opts(o.improved, o.noniso, o.e_clamp, 0, o.eps2, o.e_tau, o.g_guard,
                                          o.gravity, o.cp))
    lib().emu_solve(ct.byref(a), int(mixed), K, lds, ncu)
    return out, g
