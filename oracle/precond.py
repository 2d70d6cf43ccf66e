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
    """rho_cut: the level-cut threshold of the multigrid hierarchies (the
    inner inverses are approximations; the cut rule is a reading, see
    multigrid.cut_level)."""

    def __init__(self, M, K, C, prm, n, inner="exact", rho_cut=mg.RHO_CUT, box_length=None, cube_length=None,
                 cube_box=False, **mgkw):
        self.M = M
        self.L = (M + prm.tau * C).tocsr() if C is not None else M.tocsr()
        self.X = matching_factor(M, K, prm)
        self.inner, self.mgkw, self.N = inner, mgkw, M.shape[0]
        if inner == "mg":
            t, g, b = prm.tau, prm.gamma, prm.beta
            dom = dict(box_length=box_length, cube_length=cube_length, cube_box=cube_box)
            self.HL = mg.Hierarchy(self.L, n, a=1.0, b=0.0, rho_cut=rho_cut, **dom)
            self.HX = mg.Hierarchy(self.X, n, a=np.sqrt(t * g / b), b=t * g, rho_cut=rho_cut, **dom)

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
    def __init__(self, A, n, prm, inner="exact", rho_cut=mg.RHO_CUT, box_length=None, cube_length=None,
                 cube_box=False, **mgkw):
        self.A, self.inner, self.mgkw = A.tocsr(), inner, mgkw
        if inner == "mg":
            self.H = mg.Hierarchy(self.A, n, a=1.0, b=prm.tau * prm.delta_v, rho_cut=rho_cut,
                                  box_length=box_length, cube_length=cube_length, cube_box=cube_box)

    def apply(self, r):
        if self.inner == "exact":
            return sparse_solve(self.A, r)
        return mg.mg_solve(self.H, r, **self.mgkw)


def pcd_matrix(M, K, Cw, prm, Mrho=None):
    """A_p = (rho/tau) M_p + eta K_p + N_p(w): the convection-diffusion operator
    of the velocity block discretised on the pressure space (Mrho / tau, the
    density-weighted P1 mass, for variable density)."""
    mass = (prm.rho / prm.tau) * M if Mrho is None else Mrho / prm.tau
    A = mass + prm.viscosity * K
    if Cw is not None:
        A = A + Cw
    return A.tocsr()


class NSPreconditioner:
    """diag(A^, S^) for eq. (linearnav): A^ = diag(A_xx^{-1}, A_yy^{-1}) (the
    component blocks of the velocity operator), S^{-1} = M_p^{-1} A_p K_p^{-1}
    with K_p^{-1} on mean-zero pressures."""

    def __init__(self, Avel, M, K, Ap, prm, n, inner="exact", **mgkw):
        N2 = 4 * n * n
        self.Axx = Avel[:N2, :N2].tocsr()
        self.Ayy = Avel[N2:, N2:].tocsr()
        self.M, self.K, self.Ap = M.tocsr(), K.tocsr(), Ap.tocsr()
        self.inner, self.mgkw, self.N2, self.N = inner, mgkw, N2, n * n
        if inner == "mg":
            a, b = prm.rho / prm.tau, 1.5 * prm.viscosity
            self.Hx = mg.Hierarchy(self.Axx, n, a=a, b=b, p2=True)
            self.Hy = mg.Hierarchy(self.Ayy, n, a=a, b=b, p2=True)
            self.HK = mg.Hierarchy(self.K, n, a=0.0, b=1.0, singular=True)
            self.HM = mg.Hierarchy(self.M, n, a=1.0, b=0.0)

    def _kp_inv(self, r):
        r = r - r.mean()
        if self.inner == "mg":
            return mg.mg_solve(self.HK, r, **self.mgkw)
        N = self.N
        one = sp.csr_matrix(np.ones((N, 1)))
        B = sp.bmat([[self.K, one], [one.T, None]], format="csc")
        y = sparse_solve(B, np.concatenate([r, [0.0]]))[:N]
        return y - y.mean()

    def apply(self, r):
        N2, N = self.N2, self.N
        if self.inner == "mg":
            zx = mg.mg_solve(self.Hx, r[:N2], **self.mgkw)
            zy = mg.mg_solve(self.Hy, r[N2:2 * N2], **self.mgkw)
            zp = mg.mg_solve(self.HM, self.Ap @ self._kp_inv(r[2 * N2:]), **self.mgkw)
        else:
            zx = sparse_solve(self.Axx, r[:N2])
            zy = sparse_solve(self.Ayy, r[N2:2 * N2])
            zp = sparse_solve(self.M, self.Ap @ self._kp_inv(r[2 * N2:]))
        return np.concatenate([zx, zy, zp])
