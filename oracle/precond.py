"""Block-diagonal preconditioners of the paper (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Cahn-Hilliard (section "Iterative solvers and preconditioning", practical
preconditioner diag(L, S~)):
  L ~ M + tau C, and the matching approximation of the C = 0 Schur complement
  (tau g/beta) M + (tau g)^2 K M^{-1} K, eq. (schurCH), by
  S~ = X M^{-1} X with X = tau g K + sqrt(tau g / beta) M.
  Reading: the text prints the factor once as sqrt(tau g/beta) and once as
  sqrt(tau g/beta^2); only sqrt(tau g/beta) makes X M^{-1} X reproduce both
  terms of eq. (schurCH), so that is the one used.
  Applying S~^{-1} = X^{-1} M X^{-1}: two inner solves with X and one product
  with M.
Allen-Cahn: one inner solve with M + tau delta_v K + tau C.
Navier-Stokes: diag(A^, S^) with the pressure convection-diffusion
  approximation S^{-1} = M_p^{-1} A_p K_p^{-1} (section "Iterative solvers and
  preconditioning", last display).

Inner solves are ``exact`` (SuperLU) or ``mg`` (the cycle of ``multigrid``;
each operator a M + b K (+ c C) passes its coefficients so that the cycle is
cut at the level where it is mass-dominated).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import multigrid as mg
from .solvers import sparse_solve


def matching_factor(M, K, prm):
    t, g, b = prm.tau, prm.gamma, prm.beta
    return (t * g * K + np.sqrt(t * g / b) * M).tocsr()


def schur_exact(M, K, prm):
    """The C = 0 Schur complement of eq. (schurCH), dense (small meshes)."""
    t, g, b = prm.tau, prm.gamma, prm.beta
    Md, Kd = M.toarray(), K.toarray()
    return (t * g / b) * Md + (t * g) ** 2 * Kd @ np.linalg.solve(Md, Kd)


def schur_matching(M, K, prm):
    X = matching_factor(M, K, prm).toarray()
    return X @ np.linalg.solve(M.toarray(), X)


class CHPreconditioner:
    def __init__(self, M, K, C, prm, n, inner="exact", **mgkw):
        self.M = M
        self.L = (M + prm.tau * C).tocsr() if C is not None else M.tocsr()
        self.X = matching_factor(M, K, prm)
        self.inner, self.mgkw, self.N = inner, mgkw, M.shape[0]
        if inner == "mg":
            t, g, b = prm.tau, prm.gamma, prm.beta
            self.HL = mg.Hierarchy(self.L, n, a=1.0, b=0.0)
            self.HX = mg.Hierarchy(self.X, n, a=np.sqrt(t * g / b), b=t * g)

    def _inv(self, which, r):
        if self.inner == "exact":
            return sparse_solve(self.L if which == "L" else self.X, r)
        H = self.HL if which == "L" else self.HX
        return mg.mg_solve(H, r, **self.mgkw)

    def apply(self, r):
        N = self.N
        z1 = self._inv("L", r[:N])
        z2 = self._inv("X", self.M @ self._inv("X", r[N:]))
        return np.concatenate([z1, z2])


class ACPreconditioner:
    def __init__(self, A, n, prm, inner="exact", **mgkw):
        self.A, self.inner, self.mgkw = A.tocsr(), inner, mgkw
        if inner == "mg":
            self.H = mg.Hierarchy(self.A, n, a=1.0, b=prm.tau * prm.delta_v)

    def apply(self, r):
        if self.inner == "exact":
            return sparse_solve(self.A, r)
        return mg.mg_solve(self.H, r, **self.mgkw)
