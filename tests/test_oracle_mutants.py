"""Sensitivity of the oracle pins: plant plausible transcription mistakes in a
CPU build of the oracle source and check that the pins catch every one.

Each mutant is the oracle's C file with one textual change, compiled with gcc
into a temporary library and swapped in for the oracle while a set of pin
tests runs.  A mutant that no pin rejects would mean the pins cannot tell that
part of the oracle from a wrong version of it.  Every mutant is built twice,
as FP64 and as binary128 (the build the FP64 GPU path is checked against),
and the pins must reject both.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O
from tests import test_oracle_pins as P
from tests import test_oracle_planck as PL

MUTANTS = {
    # the typographical error of Malik et al. that the paper points out (Appendix B)
    "malik_typo_xi_for_psi": ("- L.psi * Blo + Bp * Theta)", "- L.xi * Blo + Bp * Theta)"),
    "gradient_sign_up": ("- L.psi * Blo + Bp * Theta)", "- L.psi * Blo - Bp * Theta)"),
    "gradient_sign_dn": ("- L.psi * Bup - Bp * Theta)", "- L.psi * Bup + Bp * Theta)"),
    "theta_factor_2": ("/ (2 * L.E * (1 - w * g));", "/ (L.E * (1 - w * g));"),
    "mu_star_positive": ("real ms = -mu;", "real ms = mu;"),
    "swap_G_in_dn": ("+ L.psi * L.Gm * Fb_up - (L.xi * L.Gp + L.chi * L.Gm) * Fb_lo;",
                     "+ L.psi * L.Gp * Fb_up - (L.xi * L.Gm + L.chi * L.Gp) * Fb_lo;"),
    "eps2_inverted": ("+ g0 / eps2) / D;", "+ g0 * eps2) / D;"),
    "efit_coefficient": ("K_(0.2351) * w0 * g0", "K_(0.2315) * w0 * g0"),
    "transmission_factor": ("RF(exp)(-2 * RF(sqrt)", "RF(exp)(-1 * RF(sqrt)"),
    "Pi_denominator": ("ORC_PI * (1 - w0) / (E - w0);", "ORC_PI * (1 - w0) / (E - w0 * w0);"),
    "boa_drops_beam": ("D[0] = F_boa + F_beam[0];", "D[0] = F_boa;"),
    "thomas_sign": ("for (int k = 0; k < 4; ++k) M[k] -= t[k];",
                    "for (int k = 0; k < 4; ++k) M[k] += t[k];"),
    "planck_prefactor": ("real pref = 2 * kT", "real pref = kT"),
    "beam_no_mu": ("F_beam[j] = (mu > 0) ? mu * Fstar * RF(exp)(-tau / mu) : 0;",
                   "F_beam[j] = (mu > 0) ? mu * Fstar * RF(exp)(-tau) : 0;"),
}


def pins():
    """Pin tests run against each mutant (cheap subset covering every part)."""
    yield "planck_mpmath", lambda: PL.test_planck_bin_vs_mpmath(O, 1000.0, 1e-6, 2e-6)
    yield "stefan_boltzmann", lambda: PL.test_stefan_boltzmann_partition(O, 700.0)
    for w0, g0, e in [(0.5, 0.5, 1.0832075), (0.9, 0.0, 1.0198558)]:
        yield f"efit_{w0}", lambda w0=w0, g0=g0, e=e: P.test_efit_hand_values(w0, g0, e)
    yield "absorber", lambda: P.test_pure_absorber_coefficients(0.3)
    for s in (1, 2):
        yield f"formal_{s}", lambda s=s: P.test_pure_absorption_matches_formal_solution(s)
    for s in range(8):
        yield f"ode_{s}", lambda s=s: P.test_layer_relations_solve_the_ode(s)
    for imp in (0, 1):
        yield f"dense_{imp}", lambda imp=imp: P.test_block_thomas_matches_dense_solve(0, imp)
        yield f"split_{imp}", lambda imp=imp: P.test_layer_splitting_invariance(imp, 2)
    yield "enclosure", lambda: P.test_isothermal_enclosure(0.5)
    yield "conservative", lambda: P.test_conservative_scattering_keeps_net_flux_zero(0.3)
    yield "superposition", P.test_superposition


def build_mutant(old, new, tmp, quad=False):
    src = open(O.SRC).read()
    assert src.count(old) == 1, old
    path = os.path.join(tmp, "mut.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    out = os.path.join(tmp, "libmut.so")
    extra = ["-DORC_QUAD=1"] if quad else []
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                    "-fopenmp", f"-I{O.HERE}", *extra, "-o", out, path, "-lquadmath", "-lm"],
                   check=True)
    return O.load(out)


@pytest.mark.parametrize("build", ["fp64", "binary128"])
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, build):
    old, new = MUTANTS[name]
    quad = build == "binary128"
    key = O.LIB_X if quad else O.LIB
    O.lib(quad)
    with tempfile.TemporaryDirectory() as tmp:
        mutant = build_mutant(old, new, tmp, quad)
        saved = O._libs[key]
        O._libs[key] = mutant
        caught = []
        try:
            with O.extended_build(quad):
                for pname, fn in pins():
                    try:
                        with np.errstate(all="ignore"):
                            fn()
                    except (AssertionError, ArithmeticError, ValueError, RuntimeError):
                        caught.append(pname)
        finally:
            O._libs[key] = saved
    assert caught, f"no pin rejects mutant {name} ({build})"
    print(f"{name} ({build}): rejected by {caught}")


@pytest.mark.parametrize("build", ["fp64", "binary128"])
def test_pin_subset_passes_on_the_oracle(build):
    """Control: the same pins all pass on the unmodified oracle (both builds)."""
    quad = build == "binary128"
    O.lib(quad)
    with O.extended_build(quad):
        for pname, fn in pins():
            fn()
