"""Geometric multigrid on the nested periodic P1 meshes, or on the nested
meshes of the closed square (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper approximates the inverse of each diagonal block (M + tau C, the
matching factor tau g K + sqrt(tau g / beta) M, the Allen-Cahn matrix, ...)
by a multigrid cycle (section "Iterative solvers and preconditioning"; the
numerical-results section names algebraic variants).  The GPU path uses one
geometric family on the nested right-diagonal meshes; this module writes that
cycle out plainly so the GPU cycle can be checked operation by operation.

Definition of the cycle for an operator A = a M + b K (+ c C):

* levels n, n/2, ... while the size is even and the next size is >= 4;
* prolongation P = P1 interpolation from size n/2 to n (coarse vertex (I, J)
  sits at fine vertex (2I, 2J); fine edge midpoints take the mean of the two
  coarse edge ends; the diagonal edge joins (I, J) and (I+1, J+1));
  restriction R = P^T; Galerkin coarse operators A_c = P^T A P;
* level cut: with rho_l = 8 b / (a h_l^2) (the ratio of the K and M parts of
  the diagonal; h_l = 1 / n_l on the unit square), the cycle stops at the first level with
  rho_l <= rho_cut (that operator is mass-dominated and well conditioned) or
  at the last level; a mass-dominated operator (L = M + tau C) is therefore
  handled on the fine level alone;
* smoother: Chebyshev iteration for D^{-1} A on [lmax/4, lmax] (pre and post);
  on the cut level, Chebyshev steps on [0.9 * 0.5 / (1 + rho), lmax], since the
  eigenvalues of D^{-1}(a M + b K) lie in [0.5 / (1 + rho), 2]: ``coarse``
  steps when the cut level is a coarse level, pre + post steps when the
  operator is cut on the fine level (no coarse levels at all);
* V(pre, post) cycle from a zero initial guess.

Velocity blocks (P2): the hierarchy starts with the P2 operator on mesh n and
coarsens first to P1 on the same mesh (the P1 space is a subspace of the P2
space; P interpolates P1 linearly to the edge midpoints), then follows the P1
levels above.  The P2 level smooths on [LMAX_P2/4, LMAX_P2]: for every P2
element matrix of a nonnegative combination of mass and stiffness forms the
largest eigenvalue of D_e^{-1} A_e is below 2.21, which bounds D^{-1} A.
The cut rule applies to the P1 levels; the xx/yy velocity forms have a P1
diagonal of 6 eta, so they enter with b = 1.5 eta.

Singular operators (the pressure Laplacian on the torus, constant null space):
the right-hand side is projected to mean zero, the cycle runs to the last
level, whose Chebyshev interval starts at 0.9 (1 - cos(2 pi / n_L)) / 2 (the
smallest nonzero eigenvalue of D^{-1} K there), and the result is projected to
mean zero.

The periodic cube (Kuhn tetrahedra): the same cycle on the nested meshes of
the cube (coarse vertex (I, J, K) at fine vertex (2I, 2J, 2K); a fine vertex
with odd coordinates (a, b, c) in {0, 1}^3 is the midpoint of the coarse edge
from (I, J, K) to (I + a, J + b, K + c)).  There diag(K) = 6 h and diag(M) =
0.4 h^3, so rho_l = 15 b / (a h_l^2), and D^{-1} M has spectrum in [0.5, 2.5]
(D^{-1} K in [0, 2]): the smoother's upper bound becomes LMAX_CUBE = 1.25
LMAX and the cut level's interval [0.9 * 0.5 / (1 + rho), LMAX_CUBE].

Chebyshev iteration (first kind) on [lo, hi] with theta = (hi + lo) / 2,
delta = (hi - lo) / 2, sigma = theta / delta:
  r_0 = D^{-1}(b - A x_0), d_0 = r_0 / theta, x_1 = x_0 + d_0, rho_0 = 1 / sigma;
  for i >= 1: rho_i = 1 / (2 sigma - rho_{i-1}),
              d_i = rho_i rho_{i-1} d_{i-1} + (2 rho_i / delta) D^{-1}(b - A x_i),
              x_{i+1} = x_i + d_i.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

LMAX = 2.1
LMAX_CUBE = 1.25 * LMAX
LMAX_P2 = 2.3
RHO_CUT = 0.25


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


def prolongation_box(nf: int):
    """P1 interpolation ((nf+1)^2 x (nf/2+1)^2) on the closed square: fine
    vertex (i, j) sits at (i/2, j/2) in coarse cells; with both indices even it
    is coarse vertex (i/2, j/2), otherwise the midpoint of the coarse edge that
    starts at (floor(i/2), floor(j/2)) and runs right, up or along the cell's
    diagonal."""
    nc = nf // 2
    mf, mc = nf + 1, nc + 1
    rows, cols, vals = [], [], []
    for j in range(mf):
        for i in range(mf):
            r = i + mf * j
            I, J = i // 2, j // 2
            ends = [(I, J)] if (i % 2 == 0 and j % 2 == 0) else [(I, J), (I + i % 2, J + j % 2)]
            for (a, b) in ends:
                rows.append(r)
                cols.append(a + mc * b)
                vals.append(1.0 / len(ends))
    return sp.csr_matrix((vals, (rows, cols)), shape=(mf * mf, mc * mc))


def p2_to_p1(n: int):
    """P1 on mesh n into P2 on mesh n: vertex nodes copy, edge midpoints average."""
    N = n * n
    idx = lambda i, j: (i % n) + n * (j % n)
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i, j = ii.ravel(), jj.ravel()
    rows = [np.arange(N)]
    cols = [idx(i, j)]
    vals = [np.ones(N)]
    for blk, (di, dj) in enumerate(((1, 0), (0, 1), (1, 1)), start=1):
        r = blk * N + idx(i, j)
        rows += [r, r]
        cols += [idx(i, j), idx(i + di, j + dj)]
        vals += [0.5 * np.ones(N), 0.5 * np.ones(N)]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(4 * N, N))


def prolongation_cube(nf: int):
    """P1 interpolation from the periodic cube of side nf/2 to side nf (Kuhn
    meshes, vertex (i, j, k) -> i + n j + n^2 k): each fine vertex takes the
    mean of the coarse ends of the coarse edge it halves, or copies the coarse
    vertex it sits on."""
    nc = nf // 2
    k, j, i = np.unravel_index(np.arange(nf ** 3), (nf, nf, nf))
    f = np.stack([i, j, k], 1)
    base, odd = f // 2, f % 2
    cid = lambda q: (q[:, 0] % nc) + nc * (q[:, 1] % nc) + nc * nc * (q[:, 2] % nc)
    rows = np.arange(nf ** 3)
    on_vertex = ~odd.any(axis=1)
    P = sp.coo_matrix((np.where(on_vertex, 1.0, 0.5), (rows, cid(base))), shape=(nf ** 3, nc ** 3))
    Q = sp.coo_matrix((np.where(on_vertex, 0.0, 0.5), (rows, cid(base + odd))), shape=(nf ** 3, nc ** 3))
    out = (P + Q).tocsr()
    out.eliminate_zeros()
    return out


def prolongation_cube_box(nf: int):
    """P1 interpolation between the closed cubes of side nf/2 and nf ((n+1)^3
    vertices, no identification): as prolongation_cube without wrapping."""
    nc = nf // 2
    mf, mc = nf + 1, nc + 1
    k, j, i = np.unravel_index(np.arange(mf ** 3), (mf, mf, mf))
    f = np.stack([i, j, k], 1)
    base, odd = f // 2, f % 2
    cid = lambda q: q[:, 0] + mc * q[:, 1] + mc * mc * q[:, 2]
    rows = np.arange(mf ** 3)
    on_vertex = ~odd.any(axis=1)
    P = sp.coo_matrix((np.where(on_vertex, 1.0, 0.5), (rows, cid(base))), shape=(mf ** 3, mc ** 3))
    Q = sp.coo_matrix((np.where(on_vertex, 0.0, 0.5), (rows, cid(np.minimum(base + odd, nc)))),
                      shape=(mf ** 3, mc ** 3))
    out = (P + Q).tocsr()
    out.eliminate_zeros()
    return out


def level_sizes(n: int, nmin: int = 4):
    out = [n]
    while out[-1] % 2 == 0 and out[-1] // 2 >= nmin:
        out.append(out[-1] // 2)
    return out


def rho(a, b, nl, length=1.0, cube=False):
    """r b / (a h^2) with h = length / nl, r = diag(K) h^2 / diag(M): 8 on the
    triangles, 15 on the Kuhn tetrahedra."""
    return (15.0 if cube else 8.0) * b * (nl / length) ** 2 / a


def cut_level(sizes, a, b, rho_cut=RHO_CUT, length=1.0, cube=False):
    for l, nl in enumerate(sizes):
        if rho(a, b, nl, length, cube) <= rho_cut:
            return l
    return len(sizes) - 1


class Hierarchy:
    """Galerkin hierarchy of A = a M + b K (+ c C) down to its cut level.

    ``p2``: A is a P2 operator; ``singular``: pressure Laplacian (a = 0);
    ``box_length``: A lives on the closed square [0, L]^2 (P1, (n+1)^2 nodes)
    instead of the periodic unit square; ``cube_length``: on the periodic cube
    [0, L]^3 (P1 on the Kuhn tetrahedra, n^3 nodes; with ``cube_box`` the
    closed cube, (n+1)^3 nodes)."""

    def __init__(self, A, n: int, a: float = 1.0, b: float = 0.0, nmin: int = 4,
                 rho_cut: float = RHO_CUT, p2: bool = False, singular: bool = False,
                 box_length: float | None = None, cube_length: float | None = None, cube_box: bool = False):
        if (box_length is not None or cube_length is not None) and (p2 or singular):
            raise ValueError("the closed square and the cube carry P1 operators with a mass part")
        if box_length is not None and cube_length is not None:
            raise ValueError("one domain at a time")
        sizes = level_sizes(n, nmin)
        self.singular = singular
        cube = cube_length is not None
        length = box_length if box_length is not None else (cube_length if cube else 1.0)
        lmax = LMAX_CUBE if cube else LMAX
        self.cut = len(sizes) - 1 if singular else cut_level(sizes, a, b, rho_cut, length, cube)
        self.sizes = sizes[: self.cut + 1]
        self.A = [sp.csr_matrix(A)]
        self.P = []
        self.lmax = []
        if p2:
            P = p2_to_p1(n)
            self.P.append(P)
            self.A.append(sp.csr_matrix(P.T @ self.A[-1] @ P))
            self.lmax.append(LMAX_P2)
        for nf in self.sizes[:-1]:
            if cube:
                P = prolongation_cube_box(nf) if cube_box else prolongation_cube(nf)
            else:
                P = prolongation(nf) if box_length is None else prolongation_box(nf)
            self.P.append(P)
            self.A.append(sp.csr_matrix(P.T @ self.A[-1] @ P))
            self.lmax.append(lmax)
        self.lmax.append(lmax)
        nl = self.sizes[-1]
        if singular:
            self.lo_last = 0.9 * (1.0 - np.cos(2.0 * np.pi / nl)) / 2.0
        else:
            self.lo_last = 0.9 * 0.5 / (1.0 + rho(a, b, nl, length, cube))
        self.Dinv = [1.0 / Al.diagonal() for Al in self.A]


def chebyshev(A, Dinv, b, x, lo, hi, steps):
    """``steps`` Chebyshev steps for D^{-1} A on [lo, hi] starting from x."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    rho_prev = 1.0 / sigma
    d = Dinv * (b - A @ x) / theta
    x = x + d
    for _ in range(1, steps):
        rho_i = 1.0 / (2.0 * sigma - rho_prev)
        d = rho_i * rho_prev * d + (2.0 * rho_i / delta) * (Dinv * (b - A @ x))
        x = x + d
        rho_prev = rho_i
    return x


def vcycle(H: Hierarchy, b, pre=2, post=2, coarse=8, level=0):
    A, Dinv, lmax = H.A[level], H.Dinv[level], H.lmax[level]
    x = np.zeros_like(b)
    if level == len(H.A) - 1:
        return chebyshev(A, Dinv, b, x, H.lo_last, lmax, coarse if level > 0 else pre + post)
    x = chebyshev(A, Dinv, b, x, lmax / 4.0, lmax, pre)
    r = b - A @ x
    P = H.P[level]
    x = x + P @ vcycle(H, P.T @ r, pre, post, coarse, level + 1)
    if post > 0:
        x = chebyshev(A, Dinv, b, x, lmax / 4.0, lmax, post)
    return x


def mg_solve(H: Hierarchy, b, cycles=1, **kw):
    """``cycles`` V-cycles as a stationary iteration from x = 0 (with mean-zero
    projections of the right-hand side and the result when singular)."""
    if H.singular:
        b = b - b.mean()
    x = vcycle(H, b, **kw)
    for _ in range(cycles - 1):
        x = x + vcycle(H, b - H.A[0] @ x, **kw)
    if H.singular:
        x = x - x.mean()
    return x
