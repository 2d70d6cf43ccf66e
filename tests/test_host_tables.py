"""CPU checks of the library's host-side tables (no GPU needed).

The HIP kernels index SELL-C-64 slices as ``(row >> 6) * 64 * 7 + (row & 63) + 64 k``
for the uniform 7-point P1 pattern and scatter element matrices through
per-element slot tables.  These tests read the tables the library builds
(through a host-only probe library compiled from the same source) and check
them against the oracle's CSR matrices: the pattern bit for bit, the slot
layout, the colouring, a numpy re-enactment of the coloured scatter, and the
Galerkin maps against P^T A P.
"""
import ctypes as ct
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, multigrid as mg

PROBE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2501_11767_amd", "libchns_hostprobe.so")


@pytest.fixture(scope="module")
def probe():
    if not os.path.exists(PROBE):
        pytest.skip("host probe library not built")
    L = ct.CDLL(PROBE)
    L.chns_probe_p1_nnz.restype = ct.c_int64
    return L


def _ptr(a):
    return a.ctypes.data_as(ct.c_void_p)


def _p1(probe, n):
    N = n * n
    nnz = probe.chns_probe_p1_nnz(n)
    rp = np.zeros(N + 1, np.int32)
    col = np.zeros(nnz, np.int32)
    flags = np.zeros(3, np.int32)
    probe.chns_probe_p1(n, _ptr(rp), _ptr(col), None, None, None, _ptr(flags))
    scol = np.zeros(flags[2], np.int32)
    c2s = np.zeros(nnz, np.int32)
    diag = np.zeros(N, np.int32)
    probe.chns_probe_p1(n, None, None, _ptr(scol), _ptr(c2s), _ptr(diag), None)
    return rp, col, scol, c2s, diag, flags


def _elements(probe, n):
    ne = 2 * n * n
    v = np.zeros(ne * 3, np.int32)
    p2 = np.zeros(ne * 6, np.int32)
    ty = np.zeros(ne, np.int32)
    cp = np.zeros(9, np.int32)
    probe.chns_probe_elements(n, _ptr(v), _ptr(p2), _ptr(ty), _ptr(cp))
    return v.reshape(ne, 3), p2.reshape(ne, 6), ty, cp


@pytest.mark.parametrize("n", [8, 12, 16, 32])
def test_p1_pattern_bit_exact_and_sell_layout(probe, n):
    rp, col, scol, c2s, diag, flags = _p1(probe, n)
    ref = fem.p1_mass(fem.Mesh(n))
    assert np.array_equal(rp, ref.indptr) and np.array_equal(col, ref.indices)
    assert flags[0] == 1 and flags[1] == 7
    N = n * n
    # entry k of every row sits at neighbour offset k (self, (-1,-1), (0,-1),
    # (-1,0), (1,0), (0,1), (1,1)) of the periodic mesh, vertex i + n j
    di = [0, -1, 0, -1, 1, 0, 1]
    dj = [0, -1, -1, 0, 0, 1, 1]
    rows = np.repeat(np.arange(N), 7)
    ri, rj = rows % n, rows // n
    ci, cj = col % n, col // n
    oi = (ci - ri + n + 1) % n - 1
    oj = (cj - rj + n + 1) % n - 1
    table = {(a, b): t for t, (a, b) in enumerate(zip(di, dj))}
    k = np.array([table[(a, b)] for a, b in zip(oi, oj)])
    slot = (rows >> 6) * 448 + (rows & 63) + 64 * k
    assert np.array_equal(c2s, slot)
    assert np.array_equal(scol[slot], col)
    assert np.array_equal(scol[diag], np.arange(N))
    # the stored columns follow the closed form the stencil kernels compute
    r = np.arange(N)
    i, j = r % n, r // n
    for t in range(7):
        expect = (i + di[t]) % n + n * ((j + dj[t]) % n)
        assert np.array_equal(scol[(r >> 6) * 448 + (r & 63) + 64 * t], expect), t


@pytest.mark.parametrize("n", [8, 16])
def test_colouring_is_conflict_free(probe, n):
    v, p2, ty, cp = _elements(probe, n)
    assert cp[0] == 0 and cp[8] == 2 * n * n
    for c in range(8):
        vv = v[cp[c]:cp[c + 1]].ravel()
        assert len(np.unique(vv)) == len(vv), "two triangles of one colour share a vertex"
        pp = p2[cp[c]:cp[c + 1]].ravel()
        assert len(np.unique(pp)) == len(pp), "two triangles of one colour share a P2 node"
        assert np.all(ty[cp[c]:cp[c + 1]] == c // 4)


def test_elements_match_oracle_mesh(probe):
    n = 8
    v, p2, ty, cp = _elements(probe, n)
    m = fem.Mesh(n)
    ref = {tuple(t): tuple(q) for t, q in zip(m.tri.tolist(), m.tri2.tolist())}
    assert len(ref) == len(v)
    for t, q in zip(v.tolist(), p2.tolist()):
        assert ref[tuple(t)] == tuple(q)


def _w_table():
    # int psi_k lambda_a / |T| (the table in the convection kernel)
    W = np.zeros((6, 3))
    for k in range(3):
        for a in range(3):
            W[k, a] = 1 / 30 if k == a else -1 / 60
    for e in range(3):
        for a in range(3):
            W[3 + e, a] = 1 / 15 if e == a else 2 / 15
    return W


@pytest.mark.parametrize("n", [8, 16])
def test_coloured_scatter_reenactment_matches_oracle(probe, n):
    """Re-enact the assembly kernel (element geometry from the type, the
    closed-form P2-P1 table, scatter through the slot tables) in numpy."""
    rp, col, scol, c2s, diag, flags = _p1(probe, n)
    v, p2, ty, cp = _elements(probe, n)
    N = n * n
    h = 1.0 / n
    # slot table as built by the library: slot of (v[a], v[b])
    csr = sp.csr_matrix((np.arange(len(col)), col, rp), shape=(N, N))
    from paper_2501_11767_amd import inputs
    vel = inputs.stream_velocity(n, 3, amp=0.2)
    W = _w_table()
    vals = {k: np.zeros(flags[2]) for k in ("M", "K", "C")}
    for e in range(len(v)):
        if ty[e] == 0:
            x1, y1, x2, y2 = h, 0.0, h, h
        else:
            x1, y1, x2, y2 = h, h, 0.0, h
        det = x1 * y2 - x2 * y1
        area = 0.5 * abs(det)
        g = np.zeros((3, 2))
        g[1] = (y2 / det, -x2 / det)
        g[2] = (-y1 / det, x1 / det)
        g[0] = -g[1] - g[2]
        Me = area / 12 * (np.ones((3, 3)) + np.eye(3))
        Ke = area * g @ g.T
        Va = W.T @ np.stack([vel[0][p2[e]], vel[1][p2[e]]], 1)  # (3, 2)
        Ce = area * Va @ g.T
        for a in range(3):
            for b in range(3):
                s = c2s[csr[v[e, a], v[e, b]]]
                vals["M"][s] += Me[a, b]
                vals["K"][s] += Ke[a, b]
                vals["C"][s] += Ce[a, b]
    m = fem.Mesh(n)
    for key, A in (("M", fem.p1_mass(m)), ("K", fem.p1_stiffness(m)), ("C", fem.p1_convection(m, vel))):
        got = vals[key][c2s]
        assert np.allclose(got, A.data, rtol=1e-12, atol=1e-14 * np.abs(A.data).max()), key


@pytest.mark.parametrize("nf", [8, 16, 32])
def test_galerkin_map_equals_ptap(probe, nf):
    m = fem.Mesh(nf)
    from paper_2501_11767_amd import inputs
    C = fem.p1_convection(m, inputs.stream_velocity(nf, 5, amp=0.3))
    A = (fem.p1_mass(m) + 0.3 * fem.p1_stiffness(m) + C).tocsr()
    A.sort_indices()
    P = mg.prolongation(nf)
    ref = (P.T @ A @ P).tocsr()
    ref.sort_indices()
    nc = nf // 2
    ref_pat = fem.p1_mass(fem.Mesh(nc))
    out = np.zeros(7 * nc * nc)
    assert probe.chns_probe_galerkin(nf, _ptr(np.ascontiguousarray(A.data)), _ptr(out)) == 0
    dense_ref = ref.toarray()
    got = sp.csr_matrix((out, ref_pat.indices, ref_pat.indptr), shape=(nc * nc, nc * nc)).toarray()
    assert np.allclose(got, dense_ref, rtol=1e-13, atol=1e-15 * np.abs(dense_ref).max())


@pytest.mark.parametrize("nf", [8, 16])
def test_prolongation_equals_oracle(probe, nf):
    rp = np.zeros(nf * nf + 1, np.int32)
    nnz = probe.chns_probe_prolongation(nf, _ptr(rp), None, None, None)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz)
    flags = np.zeros(4, np.int32)
    probe.chns_probe_prolongation(nf, _ptr(rp), _ptr(col), _ptr(val), _ptr(flags))
    P = sp.csr_matrix((val, col, rp), shape=(nf * nf, nf * nf // 4)).toarray()
    assert np.array_equal(P, mg.prolongation(nf).toarray())
    assert flags[1] == 2 and flags[3] == 7 and flags[2] == 1
