"""Local free-energy densities and their derivatives (FP64, nodal).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Interpolation between liquid and gas: p(Phi) = Phi^2 (3 - 2 Phi)
  (section "Free energy functional").
* Binary workloads: the double-well phi1^2 phi2^2 for the liquid and the mixing
  form phi1^2 + phi2^2 for the gas, both from section "Phase separation and
  evaporation", with phi1 = phi, phi2 = 1 - phi; without a vapour field the
  density is the double-well alone.
* Ternary workloads: the fitted quartic of eq. (appPotential) with air set to
  zero and solvent eliminated, phi_s = 1 - phi_p - phi_N; chemical potentials
  are derivatives of that reduced density.
"""
from __future__ import annotations

import numpy as np


def interp(Phi):
    return Phi * Phi * (3.0 - 2.0 * Phi)


def interp_d(Phi):
    return 6.0 * Phi * (1.0 - Phi)


# ----- binary


def f_liq_bin(phi):
    return phi ** 2 * (1.0 - phi) ** 2


def f_gas_bin(phi):
    return phi ** 2 + (1.0 - phi) ** 2


def f_bin(phi, Phi=None):
    if Phi is None:
        return f_liq_bin(phi)
    p = interp(Phi)
    return (1.0 - p) * f_liq_bin(phi) + p * f_gas_bin(phi)


def dfdphi_bin(phi, Phi=None):
    dliq = 2.0 * phi * (1.0 - phi) ** 2 - 2.0 * phi ** 2 * (1.0 - phi)
    if Phi is None:
        return dliq
    dgas = 2.0 * phi - 2.0 * (1.0 - phi)
    p = interp(Phi)
    return (1.0 - p) * dliq + p * dgas


def dfdPhi_bin(phi, Phi):
    return interp_d(Phi) * (f_gas_bin(phi) - f_liq_bin(phi))


# ----- ternary (fitted quartic, air = 0, solvent eliminated)


def _ter_parts(pp, pn):
    ps = 1.0 - pp - pn
    liq = 3.5 * pp ** 2 * pn ** 2 + 0.3 * ps ** 2
    gas = 3.5 * pp ** 2 + 3.5 * pn ** 2 + 2.0 * ps ** 2
    return ps, liq, gas


def f_ter(pp, pn, Phi):
    _, liq, gas = _ter_parts(pp, pn)
    p = interp(Phi)
    return (1.0 - p) * liq + p * gas


def dfdphi_ter(pp, pn, Phi):
    """(d f_red / d phi_p, d f_red / d phi_N); d phi_s / d phi_i = -1."""
    ps = 1.0 - pp - pn
    p = interp(Phi)
    dp = (1.0 - p) * (7.0 * pp * pn ** 2 - 0.6 * ps) + p * (7.0 * pp - 4.0 * ps)
    dn = (1.0 - p) * (7.0 * pp ** 2 * pn - 0.6 * ps) + p * (7.0 * pn - 4.0 * ps)
    return dp, dn


def dfdphis_ter(ps, Phi):
    """d f / d phi_s of the unreduced density at phi_a = 0 (for the closure of
    the eliminated phase's chemical potential)."""
    p = interp(Phi)
    return (1.0 - p) * 0.6 * ps + p * 4.0 * ps


def dfdPhi_ter(pp, pn, Phi):
    _, liq, gas = _ter_parts(pp, pn)
    return interp_d(Phi) * (gas - liq)
