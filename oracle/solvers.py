"""Direct solvers for the step systems (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method's result is the exact solution of each linear system; the Krylov
method and its preconditioner only reach it faster (section "Iterative solvers
and preconditioning").  So the oracle solves directly:

* dense LU (numpy) for small meshes,
* SuperLU (scipy.sparse.linalg.splu) up to a few hundred thousand unknowns,
* for the convection-free periodic systems, one small solve per Fourier mode:
  on the uniform periodic right-diagonal mesh M and K are block-circulant,
  with symbols written out below from their 7-point stencils.
* the Oseen saddle point with mean-zero pressure (the L^2_0 pressure space of
  the weak form) by bordering with the constraint 1^T M_p p = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def dense_solve(A, b):
    return np.linalg.solve(A.toarray(), b)


def sparse_solve(A, b):
    return spla.splu(sp.csc_matrix(A)).solve(b)


# ---------------------------------------------------------------- Fourier symbols


def p1_symbols(n: int):
    """Eigenvalues of K and M per mode, arrays indexed [ky, kx].

    K stencil: centre 4, axis neighbours -1 (diagonal couplings vanish on the
    right-diagonal mesh) -> 4 - 2 cos tx - 2 cos ty.
    M stencil: h^2/12 * (6 at the centre, 1 at the six neighbours
    (+-1,0), (0,+-1), (1,1), (-1,-1)) -> h^2/12 (6 + 2 cos tx + 2 cos ty + 2 cos(tx+ty)).
    """
    h = 1.0 / n
    t = 2.0 * np.pi * np.arange(n) / n
    ty, tx = np.meshgrid(t, t, indexing="ij")
    Khat = 4.0 - 2.0 * np.cos(tx) - 2.0 * np.cos(ty)
    Mhat = h * h / 12.0 * (6.0 + 2.0 * np.cos(tx) + 2.0 * np.cos(ty) + 2.0 * np.cos(tx + ty))
    return Khat, Mhat


def _fft(v, n):
    return np.fft.fft2(v.reshape(n, n))


def _ifft(V, n):
    return np.real(np.fft.ifft2(V)).ravel()


def fft_ch_solve(n, prm, b1, b2):
    """Per-mode 2x2 solve of eq. (CH_linear) with C = 0."""
    Kh, Mh = p1_symbols(n)
    t, g, b = prm.tau, prm.gamma, prm.beta
    a11, a12, a22 = Mh, t * g * Kh, -(t * g / b) * Mh
    B1, B2 = _fft(b1, n), _fft(b2, n)
    det = a11 * a22 - a12 * a12
    X1 = (a22 * B1 - a12 * B2) / det
    X2 = (a11 * B2 - a12 * B1) / det
    return _ifft(X1, n), _ifft(X2, n)


def fft_ac_solve(n, prm, b):
    Kh, Mh = p1_symbols(n)
    return _ifft(_fft(b, n) / (Mh + prm.tau * prm.delta_v * Kh), n)


def fft_mass_solve(n, b):
    _, Mh = p1_symbols(n)
    return _ifft(_fft(b, n) / Mh, n)


# ---------------------------------------------------------------- saddle point


def bordered_oseen_solve(Avel, B, Mp, rhs_v, dense=False, fixed=None):
    """Solve [[A, B^T, 0], [B, 0, m], [0, m^T, 0]] [v; p; lam] = [rhs_v; 0; 0]
    with m = M_p 1, giving the mean-zero pressure solution.  fixed: boolean
    mask of velocity unknowns held at zero (no-slip walls): the system is
    solved on the others and the fixed ones are returned as zeros."""
    if fixed is not None:
        free = np.flatnonzero(~fixed)
        Af = sp.csr_matrix(Avel)[free][:, free]
        Bf = sp.csr_matrix(B)[:, free]
        vf, p, lam = bordered_oseen_solve(Af, Bf, Mp, rhs_v[free], dense)
        v = np.zeros(Avel.shape[0])
        v[free] = vf
        return v, p, lam
    nv, npr = Avel.shape[0], B.shape[0]
    m = Mp @ np.ones(npr)
    mcol = sp.csr_matrix(m.reshape(-1, 1))
    K = sp.bmat([[Avel, B.T, None], [B, None, mcol], [None, mcol.T, None]], format="csc")
    rhs = np.concatenate([rhs_v, np.zeros(npr + 1)])
    x = np.linalg.solve(K.toarray(), rhs) if dense else spla.splu(K).solve(rhs)
    return x[:nv], x[nv:nv + npr], x[-1]
