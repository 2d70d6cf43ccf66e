"""Plain FP64 finite-element assembly on the periodic uniform triangulation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's discretisation section: shape-regular triangulation,
continuous P1 for volume fractions, potentials, vapour field and pressure,
Taylor-Hood P2 vector velocity; the matrices M, K, C of the Cahn-Hilliard
discretisation and J, K_sym, B of the Navier-Stokes discretisation (section
"Iterative solvers and preconditioning", definitions after eq. (matrixns)).

Mesh reading: unit square, n cells per side, periodic in x and y; cell (i, j)
is split by its (i,j)-(i+1,j+1) diagonal into a lower triangle
((i,j), (i+1,j), (i+1,j+1)) and an upper triangle ((i,j), (i+1,j+1), (i,j+1)).
Vertex (i, j) has id i + n*j.  P2 nodes: vertices, then midpoints of the
horizontal, vertical and diagonal edges, each block numbered i + n*j.

Every element integral uses the 7-point degree-5 Radon rule, which is exact
for all integrands assembled here (degree <= 5), so the values do not depend
on the rule.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# ---------------------------------------------------------------- quadrature


def radon7():
    """Degree-5 7-point rule on a triangle: barycentric points (7, 3) and
    weights (7,) normalised to sum 1 (multiply by the area)."""
    s = np.sqrt(15.0)
    a1, b1, w1 = (9 - 2 * s) / 21, (6 + s) / 21, (155 + s) / 1200
    a2, b2, w2 = (9 + 2 * s) / 21, (6 - s) / 21, (155 - s) / 1200
    pts = [(1 / 3, 1 / 3, 1 / 3),
           (a1, b1, b1), (b1, a1, b1), (b1, b1, a1),
           (a2, b2, b2), (b2, a2, b2), (b2, b2, a2)]
    w = [9 / 40, w1, w1, w1, w2, w2, w2]
    return np.array(pts), np.array(w)


QP, QW = radon7()


def p1_basis(lam):
    """P1 basis values at barycentric points: (nq, 3)."""
    return lam.copy()


def p2_basis(lam):
    """P2 basis values (nq, 6): vertices 0..2, then edge nodes 3 = (1,2),
    4 = (0,2), 5 = (0,1)."""
    l0, l1, l2 = lam[:, 0], lam[:, 1], lam[:, 2]
    return np.stack([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                     4 * l1 * l2, 4 * l0 * l2, 4 * l0 * l1], axis=1)


def p2_basis_dlam(lam):
    """d psi_k / d lambda_a at the points: (nq, 6, 3)."""
    nq = lam.shape[0]
    d = np.zeros((nq, 6, 3))
    for k in range(3):
        d[:, k, k] = 4 * lam[:, k] - 1
    d[:, 3, 1], d[:, 3, 2] = 4 * lam[:, 2], 4 * lam[:, 1]
    d[:, 4, 0], d[:, 4, 2] = 4 * lam[:, 2], 4 * lam[:, 0]
    d[:, 5, 0], d[:, 5, 1] = 4 * lam[:, 1], 4 * lam[:, 0]
    return d


# ---------------------------------------------------------------- mesh


def _geometry(m):
    """Element areas and barycentric gradients from m.xy (ne, 3, 2)."""
    x0 = m.xy[:, 0, :]
    T = np.stack([m.xy[:, 1, :] - x0, m.xy[:, 2, :] - x0], axis=2)  # columns
    det = T[:, 0, 0] * T[:, 1, 1] - T[:, 0, 1] * T[:, 1, 0]
    m.area = 0.5 * np.abs(det)
    Tinv = np.linalg.inv(T)  # rows = grad lambda_1, grad lambda_2
    g = np.zeros((m.ne, 3, 2))
    g[:, 1, :] = Tinv[:, 0, :]
    g[:, 2, :] = Tinv[:, 1, :]
    g[:, 0, :] = -g[:, 1, :] - g[:, 2, :]
    m.grad = g  # grad lambda_a per element (ne, 3, 2)


class BoxMesh:
    """Right-diagonal triangulation of the square [0, L]^2 without
    identification (the paper's closed domain, section "Numerical results"):
    (n + 1)^2 vertices numbered i + (n + 1) j, cells (i, j) split along their
    (i, j)-(i+1, j+1) diagonal like the periodic mesh.  The P1 forms assembled
    on it carry the natural (no-flux) boundary conditions of the phase
    fields and chemical potentials (eq. (bc)).

    P2 nodes in four blocks of N = (n + 1)^2 ids, each numbered i + (n + 1) j:
    the vertices, then the midpoints of the edges (i,j)-(i+1,j) (i < n), of
    (i,j)-(i,j+1) (j < n) and of (i,j)-(i+1,j+1) (i, j < n); the ids the
    ranges leave out (4n + 3 of them) belong to no element.  p2_fixed marks
    them and the wall nodes: the velocity's no-slip set (eq. (bc))."""

    def __init__(self, n: int, length: float = 1.0):
        if n < 2:
            raise ValueError("need n >= 2")
        self.n, self.length = n, length
        self.h = length / n
        m = n + 1
        self.nv = m * m
        jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        i, j = ii.ravel(), jj.ravel()
        idx = lambda a, b: a + m * b
        a, b, c, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
        lo, up = np.stack([a, b, c], 1), np.stack([a, c, d], 1)
        base = np.stack([i, j], 1).astype(np.float64)
        lo_off = base[:, None, :] + np.array([[0, 0], [1, 0], [1, 1]], dtype=np.float64)
        up_off = base[:, None, :] + np.array([[0, 0], [1, 1], [0, 1]], dtype=np.float64)
        self.tri = np.stack([lo, up], 1).reshape(-1, 3).astype(np.int64)
        N = self.nv
        H = lambda p, q: N + idx(p, q)
        V = lambda p, q: 2 * N + idx(p, q)
        D = lambda p, q: 3 * N + idx(p, q)
        # lower (a, b, c): edges (b,c) = V(i+1,j), (a,c) = D(i,j), (a,b) = H(i,j);
        # upper (a, c, d): edges (c,d) = H(i,j+1), (a,d) = V(i,j), (a,c) = D(i,j)
        lo2 = np.stack([a, b, c, V(i + 1, j), D(i, j), H(i, j)], 1)
        up2 = np.stack([a, c, d, H(i, j + 1), V(i, j), D(i, j)], 1)
        self.tri2 = np.stack([lo2, up2], 1).reshape(-1, 6).astype(np.int64)
        self.xy = np.stack([lo_off, up_off], 1).reshape(-1, 3, 2) * self.h
        self.ne = self.tri.shape[0]
        _geometry(self)

    def p2_xy(self):
        """(4N, 2) coordinates of the P2 ids (an unused id gets the point its
        formula names, outside the square or on an edge that does not exist)."""
        v = self.vertex_xy()
        h = self.h
        return np.concatenate([v, v + [0.5 * h, 0.0], v + [0.0, 0.5 * h], v + [0.5 * h, 0.5 * h]], axis=0)

    def p2_fixed(self):
        """(4N,) True for the P2 ids of the no-slip set: nodes on the walls and
        the unused ids."""
        n, m = self.n, self.n + 1
        jj, ii = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        i, j = ii.ravel(), jj.ravel()
        wall_v = (i == 0) | (i == n) | (j == 0) | (j == n)
        used = np.zeros(4 * self.nv, bool)
        used[self.tri2.ravel()] = True
        fixed = ~used
        fixed[:self.nv] |= wall_v
        fixed[self.nv:2 * self.nv] |= (j == 0) | (j == n)        # horizontal edges on the walls
        fixed[2 * self.nv:3 * self.nv] |= (i == 0) | (i == n)    # vertical edges on the walls
        return fixed

    def quad_points(self):
        return np.einsum("qa,ead->eqd", QP, self.xy)

    def vertex_xy(self):
        """(nv, 2) vertex coordinates in id order."""
        jj, ii = np.meshgrid(np.arange(self.n + 1), np.arange(self.n + 1), indexing="ij")
        return np.stack([ii.ravel(), jj.ravel()], 1) * self.h


def top_edge_load(m: BoxMesh, g=None):
    """b_i = int_{y = L} g phi_i ds over the top edge of the closed square for
    a callable g(x) (constant 1 when None), by two-point Gauss on each of its
    n segments (exact for g linear)."""
    n, h = m.n, m.h
    b = np.zeros(m.nv)
    t = 0.5 * np.array([1.0 - 1.0 / np.sqrt(3.0), 1.0 + 1.0 / np.sqrt(3.0)])
    for i in range(n):
        left, right = i + (n + 1) * n, i + 1 + (n + 1) * n
        for s in t:
            x = (i + s) * h
            w = 0.5 * h * (1.0 if g is None else g(x))
            b[left] += w * (1.0 - s)
            b[right] += w * s
    return b


class Mesh:
    """Periodic right-diagonal triangulation of the unit square."""

    def __init__(self, n: int):
        if n < 4:
            raise ValueError("need n >= 4 so that the 7-point neighbourhoods are distinct")
        self.n = n
        self.h = 1.0 / n
        N = n * n
        self.nv = N
        jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        i, j = ii.ravel(), jj.ravel()  # cell (i, j) in order i + n*j
        idx = lambda a, b: (a % n) + n * (b % n)
        a, b, c, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
        H = lambda p, q: N + idx(p, q)
        V = lambda p, q: 2 * N + idx(p, q)
        D = lambda p, q: 3 * N + idx(p, q)
        # lower (a, b, c): edge nodes (b,c) = V(i+1,j), (a,c) = D(i,j), (a,b) = H(i,j)
        lo = np.stack([a, b, c], 1)
        lo2 = np.stack([a, b, c, V(i + 1, j), D(i, j), H(i, j)], 1)
        # upper (a, c, d): edge nodes (c,d) = H(i,j+1), (a,d) = V(i,j), (a,c) = D(i,j)
        up = np.stack([a, c, d], 1)
        up2 = np.stack([a, c, d, H(i, j + 1), V(i, j), D(i, j)], 1)
        base = np.stack([i, j], 1).astype(np.float64)
        lo_off = base[:, None, :] + np.array([[0, 0], [1, 0], [1, 1]], dtype=np.float64)
        up_off = base[:, None, :] + np.array([[0, 0], [1, 1], [0, 1]], dtype=np.float64)
        # interleave: element 2*cell = lower, 2*cell + 1 = upper
        self.tri = np.stack([lo, up], 1).reshape(-1, 3).astype(np.int64)
        self.tri2 = np.stack([lo2, up2], 1).reshape(-1, 6).astype(np.int64)
        self.xy = np.stack([lo_off, up_off], 1).reshape(-1, 3, 2) * self.h
        self.ne = self.tri.shape[0]
        _geometry(self)

    def quad_points(self):
        """Physical quadrature points (ne, nq, 2), unwrapped."""
        return np.einsum("qa,ead->eqd", QP, self.xy)


def _csr(rows, cols, vals, shape):
    A = sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=shape).tocsr()
    A.sort_indices()
    return A


def _scatter(mesh_rows, mesh_cols, Ae, shape):
    """Scatter element matrices Ae (ne, r, c) with local->global maps."""
    R = np.broadcast_to(mesh_rows[:, :, None], Ae.shape)
    C = np.broadcast_to(mesh_cols[:, None, :], Ae.shape)
    return _csr(R, C, Ae, shape)


# ---------------------------------------------------------------- P1 matrices


def p1_mass(m: Mesh):
    """M_ij = int phi_j phi_i (P1)."""
    phi = p1_basis(QP)
    Ae = np.einsum("e,q,qa,qb->eab", m.area, QW, phi, phi)
    return _scatter(m.tri, m.tri, Ae, (m.nv, m.nv))


def p1_stiffness(m: Mesh):
    """K_ij = int grad phi_j . grad phi_i (P1)."""
    Ae = np.einsum("e,ead,ebd->eab", m.area, m.grad, m.grad)
    return _scatter(m.tri, m.tri, Ae, (m.nv, m.nv))


def _p2_field_at_q(m: Mesh, u_p2):
    """Evaluate a scalar P2 nodal field at the quadrature points: (ne, nq)."""
    psi = p2_basis(QP)
    return np.einsum("qk,ek->eq", psi, u_p2[m.tri2])


def p1_convection(m: Mesh, vel_p2, w_const=None):
    """C_ij = int (w . grad phi_j) phi_i with w = P2 field vel_p2 (2, 4N)
    plus an optional elementwise-constant vector w_const (ne, 2)."""
    phi = p1_basis(QP)
    wq = np.stack([_p2_field_at_q(m, vel_p2[0]), _p2_field_at_q(m, vel_p2[1])], axis=2)  # (ne,nq,2)
    if w_const is not None:
        wq = wq + w_const[:, None, :]
    # (w . grad phi_b) at q, times phi_a
    wg = np.einsum("eqd,ebd->eqb", wq, m.grad)
    Ae = np.einsum("e,q,qa,eqb->eab", m.area, QW, phi, wg)
    return _scatter(m.tri, m.tri, Ae, (m.nv, m.nv))


def p1_load(m: Mesh, f):
    """b_i = int f phi_i for a callable f(x, y), by the 7-point rule."""
    X = m.quad_points()
    fq = f(X[..., 0], X[..., 1])
    phi = p1_basis(QP)
    be = np.einsum("e,q,eq,qa->ea", m.area, QW, fq, phi)
    b = np.zeros(m.nv)
    np.add.at(b, m.tri.ravel(), be.ravel())
    return b


def p1_grad(m: Mesh, u):
    """Elementwise-constant gradient of a P1 field: (ne, 2)."""
    return np.einsum("ea,ead->ed", u[m.tri], m.grad)


# ---------------------------------------------------------------- P2 / Taylor-Hood


def _p2_grads(m: Mesh):
    """Physical gradients of the P2 basis at the points: (ne, nq, 6, 2)."""
    dl = p2_basis_dlam(QP)  # (nq, 6, 3)
    return np.einsum("qka,ead->eqkd", dl, m.grad)


def p2_mass(m: Mesh):
    """Scalar P2 mass matrix (4N x 4N)."""
    psi = p2_basis(QP)
    Ae = np.einsum("e,q,qa,qb->eab", m.area, QW, psi, psi)
    return _scatter(m.tri2, m.tri2, Ae, (4 * m.nv, 4 * m.nv))


def p2_mass_weighted(m: Mesh, rho_p1):
    """Scalar P2 mass weighted by a P1 field: int rho psi_m psi_n, rho the P1
    interpolant of the nodal values rho_p1 (degree 5: the 7-point rule is
    exact).  The variable-density mass rho^k M of eq. (matrixns)."""
    psi = p2_basis(QP)
    rq = np.einsum("qa,ea->eq", p1_basis(QP), rho_p1[m.tri])
    Ae = np.einsum("e,q,eq,qa,qb->eab", m.area, QW, rq, psi, psi)
    return _scatter(m.tri2, m.tri2, Ae, (4 * m.nv, 4 * m.nv))


def p1_mass_weighted(m: Mesh, rho_p1):
    """P1 mass weighted by a P1 field: int rho phi_i phi_j (exact)."""
    phi = p1_basis(QP)
    rq = np.einsum("qa,ea->eq", phi, rho_p1[m.tri])
    Ae = np.einsum("e,q,eq,qa,qb->eab", m.area, QW, rq, phi, phi)
    return _scatter(m.tri, m.tri, Ae, (m.nv, m.nv))


def p2_stiffness(m: Mesh):
    """Scalar P2 stiffness matrix int grad psi_j . grad psi_i."""
    G = _p2_grads(m)
    Ae = np.einsum("e,q,eqad,eqbd->eab", m.area, QW, G, G)
    return _scatter(m.tri2, m.tri2, Ae, (4 * m.nv, 4 * m.nv))


def p2_sym_stiffness(m: Mesh, eta: float):
    """K_sym for the vector P2 space ordered [x-components; y-components]:
    entry ((e,i),(c,j)) = int 2 eta sym(grad zeta_j^c) : sym(grad zeta_i^e)
    = eta int (delta_ce grad psi_i . grad psi_j + d_c psi_i d_e psi_j)."""
    G = _p2_grads(m)
    N2 = 4 * m.nv
    blocks = [[None, None], [None, None]]
    for e in range(2):
        for c in range(2):
            Ae = np.einsum("e,q,eqa,eqb->eab", m.area, QW, G[..., c], G[..., e])
            if c == e:
                Ae = Ae + np.einsum("e,q,eqad,eqbd->eab", m.area, QW, G, G)
            blocks[e][c] = _scatter(m.tri2, m.tri2, eta * Ae, (N2, N2))
    return sp.bmat(blocks, format="csr")


def p2_convection(m: Mesh, w_p2, w_const=None):
    """Scalar P2 convection J_mn = int (w . grad psi_n) psi_m, w = P2 field
    (2, 4N) plus optional elementwise constant (ne, 2)."""
    psi = p2_basis(QP)
    G = _p2_grads(m)
    wq = np.stack([_p2_field_at_q(m, w_p2[0]), _p2_field_at_q(m, w_p2[1])], axis=2)
    if w_const is not None:
        wq = wq + w_const[:, None, :]
    wg = np.einsum("eqd,eqbd->eqb", wq, G)
    Ae = np.einsum("e,q,qa,eqb->eab", m.area, QW, psi, wg)
    return _scatter(m.tri2, m.tri2, Ae, (4 * m.nv, 4 * m.nv))


def divergence_matrix(m: Mesh):
    """B (N x 8N): B_qj = - int div(zeta_j) psihat_q, pressure P1 rows,
    velocity columns [x-components; y-components]."""
    phi = p1_basis(QP)
    G = _p2_grads(m)
    N2 = 4 * m.nv
    parts = []
    for c in range(2):
        Ae = -np.einsum("e,q,qa,eqb->eab", m.area, QW, phi, G[..., c])
        parts.append(_scatter(m.tri, m.tri2, Ae, (m.nv, N2)))
    return sp.hstack(parts, format="csr")


def p2_load_vec(m: Mesh, fx, fy):
    """Vector P2 load int f . zeta for callables fx, fy: (8N,)."""
    X = m.quad_points()
    psi = p2_basis(QP)
    out = []
    for f in (fx, fy):
        fq = f(X[..., 0], X[..., 1])
        be = np.einsum("e,q,eq,qa->ea", m.area, QW, fq, psi)
        b = np.zeros(4 * m.nv)
        np.add.at(b, m.tri2.ravel(), be.ravel())
        out.append(b)
    return np.concatenate(out)


def korteweg_load(m: Mesh, grads, betas):
    """F_(c,j) = int G : grad(psi_j e_c), G = sum_i beta_i grad u_i (x) grad u_i,
    with elementwise-constant P1 gradients grads[i] (ne, 2)."""
    Gt = np.zeros((m.ne, 2, 2))
    for g, b in zip(grads, betas):
        Gt += b * np.einsum("ec,ed->ecd", g, g)
    Gp = _p2_grads(m)  # (ne, nq, 6, 2)
    intgrad = np.einsum("e,q,eqkd->ekd", m.area, QW, Gp)  # int grad psi_k
    out = []
    for c in range(2):
        be = np.einsum("ed,ekd->ek", Gt[:, c, :], intgrad)
        b = np.zeros(4 * m.nv)
        np.add.at(b, m.tri2.ravel(), be.ravel())
        out.append(b)
    return np.concatenate(out)


def p2_eval_p1_interp_mesh(m, u_p1):
    """P2 nodal values of a P1 field on any mesh with a P2 numbering (tri2):
    each element's vertex nodes take the vertex values, its edge nodes the mean
    of the edge's two vertex values (local node 3 + a is the edge opposite
    vertex a); ids that belong to no element stay 0."""
    out = np.zeros(4 * m.nv)
    t, t2 = m.tri, m.tri2
    out[t2[:, :3].ravel()] = u_p1[t].ravel()
    for a, (b, c) in zip((3, 4, 5), ((1, 2), (0, 2), (0, 1))):
        out[t2[:, a]] = 0.5 * (u_p1[t[:, b]] + u_p1[t[:, c]])
    return out


def p2_eval_p1_interp(n: int, u_p1):
    """P2 nodal values of a P1 field (vertex values copied, edge midpoints averaged)."""
    N = n * n
    idx = lambda i, j: (i % n) + n * (j % n)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i, j = i.ravel(), j.ravel()
    out = np.empty(4 * N)
    out[:N] = u_p1
    out[N:2 * N] = 0.5 * (u_p1[idx(i, j)] + u_p1[idx(i + 1, j)])
    out[2 * N:3 * N] = 0.5 * (u_p1[idx(i, j)] + u_p1[idx(i, j + 1)])
    out[3 * N:] = 0.5 * (u_p1[idx(i, j)] + u_p1[idx(i + 1, j + 1)])
    return out
