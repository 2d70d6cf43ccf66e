"""The linear systems of one semi-implicit time step (FP64, scipy.sparse).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Cahn-Hilliard, eq. (CH_linear): [[M + tau C, tau g K], [tau g K, -(tau g/beta) M]]
  with right-hand side [M phi^k; -(tau g/beta) f^k].
* Allen-Cahn (section "Iterative solvers and preconditioning", the single
  linear system after the discrete AC equation): (M + tau delta_v K + tau C) Phi
  = M Phi^k - tau gamma_v f_v^k.
* Oseen saddle point, eq. (linearnav): [[A, B^T], [B, 0]] with
  A = (rho/tau) M + J(w^k) + K_sym and right-hand side (rho/tau) M v^k + F^k.

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


def ch_matrix(M, K, C, prm: Params):
    t, g, b = prm.tau, prm.gamma, prm.beta
    A11 = M + t * C if C is not None else M
    return sp.bmat([[A11, t * g * K], [t * g * K, -(t * g / b) * M]], format="csr")


def ch_rhs(M, phi_k, fprime, prm: Params):
    t, g, b = prm.tau, prm.gamma, prm.beta
    return np.concatenate([M @ phi_k, -(t * g / b) * (M @ fprime)])


def ac_matrix(M, K, C, prm: Params):
    A = M + prm.tau * prm.delta_v * K
    if C is not None:
        A = A + prm.tau * C
    return A.tocsr()


def ac_rhs(M, Phi_k, fv, prm: Params):
    return M @ Phi_k - prm.tau * prm.gamma_v * (M @ fv)


def oseen_velocity_block(Mv, J, Ksym, prm: Params):
    """A = (rho/tau) M (per component) + J (per component) + K_sym."""
    N2 = Mv.shape[0]
    diag = (prm.rho / prm.tau) * Mv + J
    return (sp.bmat([[diag, None], [None, diag]], format="csr") + Ksym).tocsr()


def oseen_matrix(Avel, B):
    return sp.bmat([[Avel, B.T], [B, None]], format="csr")


def oseen_rhs(Mv, v_k, F, prm: Params):
    N2 = Mv.shape[0]
    mv = np.concatenate([Mv @ v_k[0], Mv @ v_k[1]])
    return np.concatenate([(prm.rho / prm.tau) * mv + F])
