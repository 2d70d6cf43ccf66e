"""Pins of the oracle's assembly against closed forms and invariants.

Every check here is independent of the oracle's own code path: monomial
integrals of the quadrature rule against the closed formula, stencils written
out by hand, the textbook P2 element mass matrix, row sums that follow from
grad 1 = 0, and consistency of the convection matrix with a smooth field.
"""
import math

import numpy as np
import pytest

from oracle import fem


def test_radon_rule_integrates_monomials_exactly():
    # int over the reference triangle of l0^a l1^b l2^c = 2|T| a! b! c! / (a+b+c+2)!
    for a in range(6):
        for b in range(6 - a):
            for c in range(6 - a - b):
                exact = 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) \
                    / math.factorial(a + b + c + 2)
                q = np.sum(fem.QW * fem.QP[:, 0] ** a * fem.QP[:, 1] ** b * fem.QP[:, 2] ** c)
                assert abs(q - exact) < 1e-15, (a, b, c)


def _stencil_cols(n, r):
    i, j = r % n, r // n
    idx = lambda a, b: (a % n) + n * (b % n)
    return sorted({idx(i, j), idx(i + 1, j), idx(i - 1, j), idx(i, j + 1), idx(i, j - 1),
                   idx(i + 1, j + 1), idx(i - 1, j - 1)})


@pytest.mark.parametrize("n", [4, 6, 8, 12])
def test_p1_pattern_closed_form(n):
    m = fem.Mesh(n)
    for A in (fem.p1_mass(m), fem.p1_stiffness(m)):
        assert A.nnz == 7 * n * n
        for r in range(n * n):
            cols = A.indices[A.indptr[r]:A.indptr[r + 1]].tolist()
            assert cols == _stencil_cols(n, r)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_p1_values_closed_form(n):
    m = fem.Mesh(n)
    M, K = fem.p1_mass(m).toarray(), fem.p1_stiffness(m).toarray()
    h2 = 1.0 / (n * n)
    idx = lambda a, b: (a % n) + n * (b % n)
    for r in [0, n + 1, n * n - 1, 3 * n + 2]:
        i, j = r % n, r // n
        assert K[r, r] == pytest.approx(4.0, abs=1e-14)
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            assert K[r, idx(i + di, j + dj)] == pytest.approx(-1.0, abs=1e-14)
        for di, dj in ((1, 1), (-1, -1)):
            assert abs(K[r, idx(i + di, j + dj)]) < 1e-14
        assert M[r, r] == pytest.approx(h2 / 2.0, rel=1e-14)
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)):
            assert M[r, idx(i + di, j + dj)] == pytest.approx(h2 / 12.0, rel=1e-14)


def test_p1_row_sums():
    n = 8
    m = fem.Mesh(n)
    M, K = fem.p1_mass(m), fem.p1_stiffness(m)
    from paper_2501_11767_amd import inputs
    vel = inputs.stream_velocity(n, 7)
    C = fem.p1_convection(m, vel)
    one = np.ones(n * n)
    assert abs(M.sum() - 1.0) < 1e-14
    assert np.abs(K @ one).max() < 1e-13
    assert np.abs(C @ one).max() < 1e-15


def test_convection_constant_velocity_is_skew_and_consistent():
    # v = (a, b) constant: C + C^T = 0 (int v.grad(uw) = 0 on the torus) and
    # C u_h ~ M (v . grad u) for smooth u at second order.
    errs = []
    a, b = 1.0, 0.5
    for n in (16, 32, 64):
        m = fem.Mesh(n)
        vel = np.zeros((2, 4 * n * n))
        vel[0], vel[1] = a, b
        C = fem.p1_convection(m, vel)
        assert np.abs((C + C.T).toarray()).max() < 1e-14
        xy = np.stack([np.arange(n * n) % n, np.arange(n * n) // n], 1) / n
        u = np.sin(2 * np.pi * xy[:, 0]) * np.cos(2 * np.pi * xy[:, 1])
        du = 2 * np.pi * (a * np.cos(2 * np.pi * xy[:, 0]) * np.cos(2 * np.pi * xy[:, 1])
                          - b * np.sin(2 * np.pi * xy[:, 0]) * np.sin(2 * np.pi * xy[:, 1]))
        M = fem.p1_mass(m)
        errs.append(np.abs(C @ u - M @ du).max() * n * n)  # scale by 1/h^2 (row weight)
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_p2_element_mass_textbook():
    # P2 mass on a triangle, times 180/|T|: vertex diag 6, vertex-vertex -1,
    # vertex with the opposite edge node -4, with an adjacent edge node 0,
    # edge diag 32, edge-edge 16.  Local order: vertices 0..2, edge nodes
    # 3=(1,2), 4=(0,2), 5=(0,1).
    ref = np.zeros((6, 6))
    for a in range(3):
        for b in range(3):
            ref[a, b] = 6 if a == b else -1
    for a in range(3):
        for e in range(3):
            ref[a, 3 + e] = ref[3 + e, a] = -4 if e == a else 0
    for e in range(3):
        for f in range(3):
            ref[3 + e, 3 + f] = 32 if e == f else 16
    psi = fem.p2_basis(fem.QP)
    loc = np.einsum("q,qa,qb->ab", fem.QW, psi, psi)  # / |T|
    assert np.allclose(loc * 180.0, ref, atol=1e-12)


@pytest.mark.parametrize("n", [4, 8])
def test_p2_and_b_patterns_and_invariants(n):
    m = fem.Mesh(n)
    Mv, Kv = fem.p2_mass(m), fem.p2_stiffness(m)
    B = fem.divergence_matrix(m)
    N = n * n
    assert Mv.nnz == 46 * N and Kv.nnz == 46 * N
    rowlen = np.diff(Mv.indptr)
    assert (rowlen[:N] == 19).all() and (rowlen[N:] == 9).all()
    assert B.nnz == 38 * N and (np.diff(B.indptr) == 38).all()
    assert abs(Mv.sum() - 1.0) < 1e-13
    assert np.abs(Kv @ np.ones(4 * N)).max() < 1e-12
    Ks = fem.p2_sym_stiffness(m, 1.3)
    for c in range(2):
        u = np.zeros(8 * N)
        u[c * 4 * N:(c + 1) * 4 * N] = 1.0
        assert np.abs(Ks @ u).max() < 1e-11
        assert np.abs(B @ u).max() < 1e-14     # div of a constant field
    assert np.abs(np.ones(N) @ B).max() < 1e-14  # int div v = 0 on the torus


def test_p2_convection_rows_sum_to_zero_and_skew_for_constant_w():
    n = 8
    m = fem.Mesh(n)
    w = np.zeros((2, 4 * n * n))
    w[0], w[1] = 0.3, -0.7
    J = fem.p2_convection(m, w)
    assert np.abs(J @ np.ones(4 * n * n)).max() < 1e-14
    assert np.abs((J + J.T).toarray()).max() < 1e-14


def test_korteweg_load_of_constant_gradient_vanishes():
    # G constant in space => int G : grad zeta = 0 for every periodic zeta.
    n = 8
    m = fem.Mesh(n)
    g = np.tile(np.array([[0.4, -0.2]]), (m.ne, 1))
    F = fem.korteweg_load(m, [g], [2.0])
    assert np.abs(F).max() < 1e-14
