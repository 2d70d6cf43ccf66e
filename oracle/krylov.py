"""Plain flexible GMRES (FP64) as a reference for the GPU Krylov engine.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves every system with GMRES and the stopping rule
||b - A z|| <= max(rtol ||b||, atol) (section "Numerical results").  The inner
multigrid solves make the preconditioner a different operator at each call in
general, so the right-preconditioned flexible variant is used: z_j = P^{-1} v_j
is stored and the update is x = x0 + Z y.  The Arnoldi basis is built with
classical Gram-Schmidt applied twice; the small least-squares problem
min || beta e1 - H y || is solved by numpy's lstsq (the GPU path uses Givens
rotations instead).
"""
from __future__ import annotations

import numpy as np


def fgmres(A, b, x0=None, prec=None, restart=30, rtol=1e-8, atol=0.0, maxiter=1000,
           fixed_iters=None):
    """Returns (x, iterations, history of true residual norms at restarts).

    ``fixed_iters``: run exactly that many Arnoldi steps in one cycle and
    return the iterate (for step-by-step comparison).
    """
    matvec = A if callable(A) else (lambda v: A @ v)
    P = prec if prec is not None else (lambda v: v)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    tol = max(rtol * bnorm, atol)
    its, hist = 0, []
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta)
        if (beta <= tol and fixed_iters is None) or its >= maxiter:
            return x, its, hist
        m = restart if fixed_iters is None else fixed_iters
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        k_done = 0
        for j in range(m):
            z = P(V[j])
            Z.append(z)
            w = matvec(z)
            for _ in range(2):
                Vm = np.array(V)
                h = Vm @ w
                w = w - Vm.T @ h
                H[: j + 1, j] += h
            H[j + 1, j] = np.linalg.norm(w)
            k_done = j + 1
            its += 1
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)
            res = np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y)
            if H[j + 1, j] == 0.0:
                break
            V.append(w / H[j + 1, j])
            if fixed_iters is None and (res <= tol or its >= maxiter):
                break
        x = x + np.array(Z[:k_done]).T @ y
        if fixed_iters is not None:
            return x, its, hist
