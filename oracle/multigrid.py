"""Geometric multigrid V-cycle on the nested periodic P1 meshes (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper approximates the inverse of each diagonal block (M + tau C, the
matching factor tau g K + sqrt(tau g / beta) M, the Allen-Cahn matrix, the
velocity block, the pressure stiffness) by a multigrid cycle (section
"Iterative solvers and preconditioning"; the numerical-results section names
algebraic variants).  The GPU path uses one geometric family on the nested
right-diagonal meshes; this module writes that cycle out plainly so the GPU
cycle can be checked operation by operation:

* levels n, n/2, ... while the size is even and the next size is >= 4;
* prolongation P = P1 interpolation from the mesh of size n/2 to size n
  (coarse vertex (I, J) sits at fine vertex (2I, 2J); fine edge midpoints take
  the mean of the two coarse edge ends; the diagonal edge joins (I, J) and
  (I+1, J+1));
* restriction R = P^T, Galerkin coarse operators A_c = P^T A P;
* smoother: damped Jacobi x <- x + omega D^{-1} (b - A x);
* V(pre, post) cycle from a zero initial guess; the coarsest level applies
  ``coarse`` damped-Jacobi sweeps.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def prolongation(nf: int):
    """P1 interpolation (nf^2 x (nf/2)^2) on the periodic right-diagonal mesh."""
    nc = nf // 2
    cid = lambda I, J: (I % nc) + nc * (J % nc)
    rows, cols, vals = [], [], []
    for J in range(nc):
        for I in range(nc):
            f = lambda i, j: (i % nf) + nf * (j % nf)
            rows.append(f(2 * I, 2 * J)); cols.append(cid(I, J)); vals.append(1.0)
            for (di, dj), (dI, dJ) in (((1, 0), (1, 0)), ((0, 1), (0, 1)), ((1, 1), (1, 1))):
                r = f(2 * I + di, 2 * J + dj)
                rows += [r, r]
                cols += [cid(I, J), cid(I + dI, J + dJ)]
                vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf * nf, nc * nc))


def level_sizes(n: int, nmin: int = 4):
    out = [n]
    while out[-1] % 2 == 0 and out[-1] // 2 >= nmin:
        out.append(out[-1] // 2)
    return out


class Hierarchy:
    def __init__(self, A, n: int, nmin: int = 4):
        self.sizes = level_sizes(n, nmin)
        self.A = [sp.csr_matrix(A)]
        self.P = []
        for nf in self.sizes[:-1]:
            P = prolongation(nf)
            self.P.append(P)
            self.A.append(sp.csr_matrix(P.T @ self.A[-1] @ P))
        self.Dinv = [1.0 / Al.diagonal() for Al in self.A]


def vcycle(H: Hierarchy, b, pre=2, post=2, coarse=16, omega=2.0 / 3.0, level=0):
    A, Dinv = H.A[level], H.Dinv[level]
    x = np.zeros_like(b)
    if level == len(H.A) - 1:
        for _ in range(coarse):
            x = x + omega * Dinv * (b - A @ x)
        return x
    for _ in range(pre):
        x = x + omega * Dinv * (b - A @ x)
    r = b - A @ x
    P = H.P[level]
    x = x + P @ vcycle(H, P.T @ r, pre, post, coarse, omega, level + 1)
    for _ in range(post):
        x = x + omega * Dinv * (b - A @ x)
    return x


def mg_solve(H: Hierarchy, b, cycles=1, **kw):
    """``cycles`` V-cycles as a stationary iteration from x = 0."""
    x = vcycle(H, b, **kw)
    for _ in range(cycles - 1):
        x = x + vcycle(H, b - H.A[0] @ x, **kw)
    return x
