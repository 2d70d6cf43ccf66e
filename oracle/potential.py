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


# ----- quaternary: eq. (appPotential) in full (polymer, NFA, solvent, air),
# the air eliminated as phi_a = 1 - phi_p - phi_N - phi_s (section "Numerical
# results")


def quaternary(pp, pn, ps, Phi):
    """Nodal terms of eq. (appPotential) with the air eliminated.  Liquid
    3.5 p^2 n^2 + 0.3 s^2 + 0.3 a^2 - 10 s a, gas 3.5 p^2 + 3.5 n^2 + 2 s^2
    + 0.1 a^2, interpolated by p(Phi).  Returns f, dp, dn, ds (derivatives along
    phi_a = 1 - phi_p - phi_N - phi_s: the unreduced partial minus the air's),
    fa (the unreduced d f / d phi_a, for the closure of mu_a) and fv."""
    pa = 1.0 - pp - pn - ps
    liq = 3.5 * pp ** 2 * pn ** 2 + 0.3 * ps ** 2 + 0.3 * pa ** 2 - 10.0 * ps * pa
    gas = 3.5 * pp ** 2 + 3.5 * pn ** 2 + 2.0 * ps ** 2 + 0.1 * pa ** 2
    l1 = [7.0 * pp * pn ** 2, 7.0 * pp ** 2 * pn, 0.6 * ps - 10.0 * pa, 0.6 * pa - 10.0 * ps]
    g1 = [7.0 * pp, 7.0 * pn, 4.0 * ps, 0.2 * pa]
    P = interp(Phi)
    F = [(1.0 - P) * l1[i] + P * g1[i] for i in range(4)]
    return dict(f=(1.0 - P) * liq + P * gas, dp=F[0] - F[3], dn=F[1] - F[3], ds=F[2] - F[3], fa=F[3],
                fv=interp_d(Phi) * (gas - liq))


# ----- ternary densities in unreduced form, with the Flory-Huggins option
#
# Section "Free energy functional": the liquid density is the Flory-Huggins
# mixing energy sum_i (phi_i / N_i) ln phi_i + sum_{i<j} chi_ij phi_i phi_j and
# the gas density sum_i phi_i ln(phi_i / phi_sat(i)), interpolated by p(Phi).
# Section "Numerical results": every phi ln phi is replaced by its Taylor
# polynomial of degree 4 about phi = 1/2, and the truncated phase fields of
# eq. (truncateCH) may be used to find the next iterates.  Here the phases are
# polymer, NFA and solvent with air set to zero (its terms are constants) and
# the solvent eliminated, phi_s = 1 - phi_p - phi_N.  The fitted quartic of
# eq. (appPotential) is written in the same unreduced form, so one chain rule
# serves both.


def xlogx_taylor_coefficients():
    """c_k = g^(k)(1/2) / k!, k = 0..4, for g(x) = x ln x: g' = ln x + 1,
    g'' = 1/x, g''' = -1/x^2, g'''' = 2/x^3."""
    h = 0.5
    derivs = [h * np.log(h), np.log(h) + 1.0, 1.0 / h, -1.0 / h ** 2, 2.0 / h ** 3]
    fact = [1.0, 1.0, 2.0, 6.0, 24.0]
    return [d / f for d, f in zip(derivs, fact)]


def xlogx_taylor4(x, deriv=0):
    """The degree-4 Taylor polynomial of x ln x about 1/2 (or its derivative
    of order `deriv` <= 2) at x."""
    c = xlogx_taylor_coefficients()
    u = x - 0.5
    if deriv == 0:
        return c[0] + u * (c[1] + u * (c[2] + u * (c[3] + u * c[4])))
    if deriv == 1:
        return c[1] + u * (2.0 * c[2] + u * (3.0 * c[3] + u * 4.0 * c[4]))
    if deriv == 2:
        return 2.0 * c[2] + u * (6.0 * c[3] + u * 12.0 * c[4])
    raise ValueError(deriv)


class Quartic:
    """Eq. (appPotential) with phi_a = 0: liquid 3.5 p^2 n^2 + 0.3 s^2, gas
    3.5 p^2 + 3.5 n^2 + 2 s^2 (p, n, s: polymer, NFA, solvent)."""

    def parts(self, p, n, s):
        z = np.zeros_like(p)
        liq = 3.5 * p ** 2 * n ** 2 + 0.3 * s ** 2
        gas = 3.5 * p ** 2 + 3.5 * n ** 2 + 2.0 * s ** 2
        liq1 = [7.0 * p * n ** 2, 7.0 * p ** 2 * n, 0.6 * s]
        gas1 = [7.0 * p, 7.0 * n, 4.0 * s]
        liq2 = [[7.0 * n ** 2, 14.0 * p * n, z], [14.0 * p * n, 7.0 * p ** 2, z], [z, z, 0.6 + z]]
        gas2 = [[7.0 + z, z, z], [z, 7.0 + z, z], [z, z, 4.0 + z]]
        return liq, gas, liq1, gas1, liq2, gas2


class FloryHuggins:
    """Flory-Huggins liquid and ideal-gas densities with x ln x replaced by its
    Taylor-4 polynomial; defaults are the paper's values for the full model
    (N_p = N_NFA = 5, N_s = 1; chi_(p,NFA) = 4, chi_(p,s) = chi_(NFA,s) = 0.3;
    phi_sat = 1e-8, 1e-8, 1e-6)."""

    def __init__(self, nsize=(5.0, 5.0, 1.0), chi=(4.0, 0.3, 0.3), phi_sat=(1e-8, 1e-8, 1e-6)):
        self.nsize, self.chi, self.phi_sat = tuple(nsize), tuple(chi), tuple(phi_sat)

    def parts(self, p, n, s):
        x = (p, n, s)
        N = self.nsize
        c_pn, c_ps, c_ns = self.chi
        L = [np.log(v) for v in self.phi_sat]
        g = [xlogx_taylor4(v) for v in x]
        g1 = [xlogx_taylor4(v, 1) for v in x]
        g2 = [xlogx_taylor4(v, 2) for v in x]
        z = np.zeros_like(p)
        liq = g[0] / N[0] + g[1] / N[1] + g[2] / N[2] + c_pn * p * n + c_ps * p * s + c_ns * n * s
        gas = g[0] + g[1] + g[2] - p * L[0] - n * L[1] - s * L[2]
        liq1 = [g1[0] / N[0] + c_pn * n + c_ps * s, g1[1] / N[1] + c_pn * p + c_ns * s,
                g1[2] / N[2] + c_ps * p + c_ns * n]
        gas1 = [g1[i] - L[i] for i in range(3)]
        liq2 = [[g2[0] / N[0], c_pn + z, c_ps + z], [c_pn + z, g2[1] / N[1], c_ns + z],
                [c_ps + z, c_ns + z, g2[2] / N[2]]]
        gas2 = [[g2[0], z, z], [z, g2[1], z], [z, z, g2[2]]]
        return liq, gas, liq1, gas1, liq2, gas2


def ternary(pp, pn, Phi, pot, truncate=False):
    """The reduced ternary density and its derivatives at the nodes.

    With truncate, the phase fields enter as clip(phi, 0, 1) (eq. (truncateCH);
    the solvent as clip(1 - phi_p - phi_N, 0, 1)), and the derivatives carry
    the clip's derivative (1 inside [0, 1], 0 outside).  Returns a dict with
    f (density), dp, dn (d f / d phi_p, d phi_N along phi_s = 1 - phi_p -
    phi_N), fv (d f / d Phi_v), fs (the unreduced d f / d phi_s, which the
    closure of the eliminated phase uses), and the second derivatives
    hpp, hpn, hnn, hpP, hnP, hvP, and hsp, hsn, hsP (of fs)."""
    ps = 1.0 - pp - pn
    if truncate:
        ind = [((v >= 0.0) & (v <= 1.0)).astype(float) for v in (pp, pn, ps)]
        x = [np.clip(v, 0.0, 1.0) for v in (pp, pn, ps)]
    else:
        ind = [np.ones_like(pp)] * 3
        x = [pp, pn, ps]
    liq, gas, l1, g1, l2, g2 = pot.parts(*x)
    P, dP, ddP = interp(Phi), interp_d(Phi), 6.0 * (1.0 - 2.0 * Phi)
    F1 = [(1.0 - P) * l1[i] + P * g1[i] for i in range(3)]
    F2 = [[(1.0 - P) * l2[i][j] + P * g2[i][j] for j in range(3)] for i in range(3)]
    D1 = [dP * (g1[i] - l1[i]) for i in range(3)]  # d F1_i / d Phi
    Ip, In, Is = ind
    # d/dphi_p of a function of (clip(p), clip(n), clip(1 - p - n)): chain rule
    out = dict(f=(1.0 - P) * liq + P * gas,
               dp=F1[0] * Ip - F1[2] * Is, dn=F1[1] * In - F1[2] * Is,
               fv=dP * (gas - liq), fs=F1[2])
    out["hpp"] = F2[0][0] * Ip - 2.0 * F2[0][2] * Ip * Is + F2[2][2] * Is
    out["hnn"] = F2[1][1] * In - 2.0 * F2[1][2] * In * Is + F2[2][2] * Is
    out["hpn"] = F2[0][1] * Ip * In - F2[0][2] * Ip * Is - F2[1][2] * In * Is + F2[2][2] * Is
    out["hpP"] = D1[0] * Ip - D1[2] * Is
    out["hnP"] = D1[1] * In - D1[2] * Is
    out["hvP"] = ddP * (gas - liq)
    out["hsp"] = F2[2][0] * Ip - F2[2][2] * Is
    out["hsn"] = F2[2][1] * In - F2[2][2] * Is
    out["hsP"] = D1[2]
    return out
