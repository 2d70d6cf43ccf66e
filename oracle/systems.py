"""The linear systems of one semi-implicit time step (FP64, scipy.sparse).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Cahn-Hilliard, eq. (CH_linear): [[M + tau C, tau g K], [tau g K, -(tau g/beta) M]]
  with right-hand side [M phi^k; -(tau g/beta) f^k].
* Allen-Cahn (section "Iterative solvers and preconditioning", the single
  linear system after the discrete AC equation): (M + tau delta_v K + tau C) Phi
  = M Phi^k - tau gamma_v f_v^k.
* Oseen saddle point, eq. (linearnav): [[A, B^T], [B, 0]] with
  A = (rho/tau) M + J(w^k) + K_sym and right-hand side (rho/tau) M v^k + F^k;
  with variable density rho^k M is the mass weighted by the P1 field rho^k.

Parameter readings: beta_i = beta_v = eps^2, gamma_i = mobility,
gamma_v = evaporation rate, delta_v = gamma_v eps^2, rho = 1, alpha_i = alpha.
Explicit terms are nodal: f^k = M f'(phi^k) evaluated at the vertices.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Params:
    eps: float
    tau: float
    mobility: float = 1.0
    evap_rate: float = 0.0
    viscosity: float = 1.0
    alpha: float = 1e-8
    rho: float = 1.0
    # ternary density: None for the fitted quartic of eq. (appPotential), or a
    # potential.FloryHuggins; truncate: potential terms at the truncated
    # phase fields of eq. (truncateCH)
    potential: object = None
    truncate: bool = False
    # variable density (eq. (matrixns)): rho^k = sum_i rho_i phi_i^k with the
    # pure densities (polymer, NFA, solvent) and phi_s = 1 - phi_p - phi_N (air
    # set to zero); None: the constant rho above
    rho_pure: tuple | None = None
    # Picard passes of the Oseen solve per step: pass m convects with the
    # velocity of pass m - 1 (pass 1 with v^k, the linear scheme); stop early
    # when the relative 2-norm change of the velocity is <= picard_tol
    picard: int = 1
    picard_tol: float = 0.0
    # evaporation at the top wall of the closed square (eq. (bc), Hertz-Knudsen
    # flux): d phi / dn = j_out = top_flux (phi^k(x_ref) - flux_inf) on the top
    # edge, x_ref its midpoint; top_flux lumps the flow rate, the square root
    # and P_0 into one coefficient
    top_flux: float = 0.0
    flux_inf: float = 0.0
    # per-phase gradient coefficients (beta_p, beta_N, beta_s, beta_a) of the
    # quaternary model (section "Numerical results" gives them per phase);
    # None: eps^2 for every phase.  The vapour field keeps beta_v = eps^2.
    betas: tuple | None = None

    def beta_of(self, i: int) -> float:
        return self.beta if self.betas is None else self.betas[i]

    @property
    def beta(self):
        return self.eps ** 2

    @property
    def gamma(self):
        return self.mobility

    @property
    def gamma_v(self):
        return self.evap_rate

    @property
    def delta_v(self):
        return self.evap_rate * self.eps ** 2

    @property
    def beta_v(self):
        return self.eps ** 2


def ch_matrix(M, K, C, prm: Params, beta=None):
    """beta: the phase's gradient coefficient (default eps^2)."""
    t, g = prm.tau, prm.gamma
    b = prm.beta if beta is None else beta
    A11 = M + t * C if C is not None else M
    return sp.bmat([[A11, t * g * K], [t * g * K, -(t * g / b) * M]], format="csr")


def ch_rhs(M, phi_k, fprime, prm: Params, flux=None, beta=None):
    """flux: the boundary load int_Gamma_t j_out w_i ds of the second CH
    equation (eq. (weakch) for mu: M mu - beta K phi = M f' - beta flux),
    which enters the scaled second row as + tau g flux.  beta: the phase's
    gradient coefficient (default eps^2)."""
    t, g = prm.tau, prm.gamma
    b = prm.beta if beta is None else beta
    second = -(t * g / b) * (M @ fprime)
    if flux is not None:
        second = second + t * g * flux
    return np.concatenate([M @ phi_k, second])


def ac_matrix(M, K, C, prm: Params):
    A = M + prm.tau * prm.delta_v * K
    if C is not None:
        A = A + prm.tau * C
    return A.tocsr()


def ac_rhs(M, Phi_k, fv, prm: Params):
    return M @ Phi_k - prm.tau * prm.gamma_v * (M @ fv)


def oseen_velocity_block(Mv, J, Ksym, prm: Params, Mrho=None):
    """A = (rho/tau) M (per component) + J (per component) + K_sym; with the
    density-weighted scalar mass Mrho (int rho^k psi_m psi_n), Mrho / tau in
    place of (rho/tau) M."""
    mass = (prm.rho / prm.tau) * Mv if Mrho is None else Mrho / prm.tau
    diag = mass + J
    return (sp.bmat([[diag, None], [None, diag]], format="csr") + Ksym).tocsr()


def oseen_matrix(Avel, B):
    return sp.bmat([[Avel, B.T], [B, None]], format="csr")


def oseen_rhs(Mv, v_k, F, prm: Params, Mrho=None):
    """(rho/tau) M v^k + F^k (Mrho v^k / tau with the density-weighted mass)."""
    if Mrho is None:
        mv = (prm.rho / prm.tau) * np.concatenate([Mv @ v_k[0], Mv @ v_k[1]])
    else:
        mv = np.concatenate([Mrho @ v_k[0], Mrho @ v_k[1]]) / prm.tau
    return mv + F


def density(prm: Params, pp, pn):
    """rho^k at the vertices: sum_i rho_i phi_i^k over polymer, NFA and the
    eliminated solvent (air zero); None for constant density."""
    if prm.rho_pure is None:
        return None
    rp, rn, rs = prm.rho_pure
    return rp * pp + rn * pn + rs * (1.0 - pp - pn)
