"""Plain FP64 P1 assembly on the periodic cube (tetrahedra).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's three-dimensional runs (section "Numerical results": uniform
triangulations of the 10 x 10 x 10 domain with linear Lagrange elements for the
phase fields and chemical potentials) in the same reading as the
two-dimensional oracle: the unit cube, n cells per side, periodic in x, y and
z.  Each cube cell (i, j, k) is split into the six tetrahedra of the Kuhn
(Freudenthal) subdivision that share the cell's main diagonal: for each
ordering (a, b, c) of the three axes the tetrahedron
    v0, v0 + e_a, v0 + e_a + e_b, v0 + (1, 1, 1),    v0 = (i, j, k).
Vertex (i, j, k) has id i + n j + n^2 k.  Every edge of this mesh runs along
one of the seven directions with components in {0, 1}, so a vertex couples to
14 neighbours.

Element integrals: the mass matrix by the exact formula
int lambda_a lambda_b = |T| (1 + delta_ab) / 20; the stiffness matrix from the
constant barycentric gradients; loads by the symmetric 4-point degree-2 rule.
"""
from __future__ import annotations

from itertools import permutations

import numpy as np
import scipy.sparse as sp

# ordering of the axes of the six tetrahedra of a cell (the library numbers its
# element types in this order)
KUHN_ORDERS = tuple(permutations(range(3)))


def kuhn_offsets():
    """(6, 4, 3) vertex offsets of the six tetrahedra of a unit cell."""
    out = []
    for a, b, c in KUHN_ORDERS:
        v = [np.zeros(3, int)]
        for ax in (a, b, c):
            w = v[-1].copy()
            w[ax] += 1
            v.append(w)
        out.append(np.stack(v))
    return np.stack(out)


class Mesh3:
    """Kuhn triangulation of the cube [0, L]^3 with n cells per side: periodic
    (n^3 vertices i + n j + n^2 k), or with ``box`` the closed cube without
    identification ((n+1)^3 vertices i + (n+1) j + (n+1)^2 k, 0 <= i, j, k <= n)."""

    def __init__(self, n: int, length: float = 1.0, box: bool = False):
        if n < (1 if box else 3):
            raise ValueError("need n >= 3 on the periodic cube (distinct neighbourhoods), n >= 1 on the closed one")
        self.n, self.length, self.box = n, length, box
        self.h = length / n
        m = n + 1 if box else n  # vertices per side
        self.m = m
        self.nv = m ** 3
        kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        base = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1)  # cell (i, j, k) in order i + n j + n^2 k
        off = kuhn_offsets()
        pts = base[:, None, None, :] + off[None, :, :, :]  # (cells, 6, 4, 3), unwrapped
        w = pts if box else pts % n
        ids = w[..., 0] + m * w[..., 1] + m * m * w[..., 2]
        self.tet = ids.reshape(-1, 4).astype(np.int64)
        self.type = np.tile(np.arange(6), base.shape[0])
        self.xyz = pts.reshape(-1, 4, 3).astype(np.float64) * self.h
        self.ne = self.tet.shape[0]
        x0 = self.xyz[:, 0, :]
        T = np.stack([self.xyz[:, a, :] - x0 for a in (1, 2, 3)], axis=2)  # columns
        det = np.linalg.det(T)
        self.vol = np.abs(det) / 6.0
        Tinv = np.linalg.inv(T)  # rows: grad lambda_1..3
        g = np.zeros((self.ne, 4, 3))
        g[:, 1:, :] = Tinv
        g[:, 0, :] = -g[:, 1:, :].sum(axis=1)
        self.grad = g

    def vertex_xyz(self):
        m = self.m
        kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
        return np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1) * self.h


def _scatter(rows, Ae, N):
    R = np.broadcast_to(rows[:, :, None], Ae.shape)
    C = np.broadcast_to(rows[:, None, :], Ae.shape)
    A = sp.coo_matrix((Ae.ravel(), (R.ravel(), C.ravel())), shape=(N, N)).tocsr()
    A.sort_indices()
    return A


def p1_mass(m: Mesh3):
    """M_ab = |T| (1 + delta_ab) / 20 per element."""
    loc = (np.ones((4, 4)) + np.eye(4)) / 20.0
    return _scatter(m.tet, m.vol[:, None, None] * loc[None], m.nv)


def p1_stiffness(m: Mesh3):
    """K_ab = |T| grad lambda_a . grad lambda_b per element."""
    Ae = np.einsum("e,ead,ebd->eab", m.vol, m.grad, m.grad)
    return _scatter(m.tet, Ae, m.nv)


def top_face_load(m: Mesh3):
    """b_i = int_{z = L} phi_i dS over the top face of the closed cube: the
    faces of the tetrahedra with three vertices on z = L, each adding a third
    of its area to each of its vertices (exact for P1)."""
    if not m.box:
        raise ValueError("the top face belongs to the closed cube")
    b = np.zeros(m.nv)
    top = np.isclose(m.xyz[..., 2], m.length)  # (ne, 4)
    for e in np.nonzero(top.sum(axis=1) == 3)[0]:
        a = np.nonzero(top[e])[0]
        p = m.xyz[e, a]
        area = 0.5 * np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[0]))
        b[m.tet[e, a]] += area / 3.0
    return b


def _rule4():
    a, b = 0.5854101966249685, 0.1381966011250105
    lam = np.full((4, 4), b)
    np.fill_diagonal(lam, a)
    return lam, np.full(4, 0.25)


def p1_load(m: Mesh3, f):
    """b_i = int f phi_i for a callable f(x, y, z), 4-point degree-2 rule."""
    lam, w = _rule4()
    X = np.einsum("qa,ead->eqd", lam, m.xyz)
    fq = f(X[..., 0], X[..., 1], X[..., 2])
    be = np.einsum("e,q,eq,qa->ea", m.vol, w, fq, lam)
    b = np.zeros(m.nv)
    np.add.at(b, m.tet.ravel(), be.ravel())
    return b
