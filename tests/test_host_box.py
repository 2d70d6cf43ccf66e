"""CPU checks of the library's host tables on the closed square [0, L]^2
(no-flux boundaries, (n+1)^2 vertices i + (n+1) j): the P1 pattern against the
oracle's, the padded SELL layout (a neighbour outside the square stored as the
row's own column), the element tables and colouring, a re-enactment of the
coloured scatter, and the nested prolongation with its Galerkin map against
the oracle's coarse-mesh forms (P^T A_h P = A_2h holds exactly for nested P1
spaces)."""
import ctypes as ct
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem

PROBE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2501_11767_amd", "libchns_hostprobe.so")
L10 = 10.0
DI = [0, -1, 0, -1, 1, 0, 1]  # neighbour order of the 7-point rows
DJ = [0, -1, -1, 0, 0, 1, 1]


@pytest.fixture(scope="module")
def probe():
    if not os.path.exists(PROBE):
        pytest.skip("host probe library not built")
    L = ct.CDLL(PROBE)
    L.chns_probe_box_p1_nnz.restype = ct.c_int64
    return L


def _ptr(a):
    return a.ctypes.data_as(ct.c_void_p)


def _p1(probe, n):
    N = (n + 1) ** 2
    nnz = probe.chns_probe_box_p1_nnz(n)
    rp = np.zeros(N + 1, np.int32)
    col = np.zeros(nnz, np.int32)
    flags = np.zeros(4, np.int32)
    probe.chns_probe_box_p1(n, _ptr(rp), _ptr(col), None, None, None, _ptr(flags))
    scol = np.zeros(flags[2], np.int32)
    c2s = np.zeros(nnz, np.int32)
    diag = np.zeros(N, np.int32)
    probe.chns_probe_box_p1(n, None, None, _ptr(scol), _ptr(c2s), _ptr(diag), None)
    return rp, col, scol, c2s, diag, flags


def _elements(probe, n):
    ne = 2 * n * n
    v = np.zeros(ne * 3, np.int32)
    ty = np.zeros(ne, np.int32)
    cp = np.zeros(9, np.int32)
    np2 = probe.chns_probe_box_elements(n, _ptr(v), _ptr(ty), _ptr(cp))
    return v.reshape(ne, 3), ty, cp, np2


@pytest.mark.parametrize("n", [8, 10, 32])
def test_pattern_and_padded_sell_layout(probe, n):
    m = fem.BoxMesh(n, L10)
    ref = fem.p1_mass(m)
    rp, col, scol, c2s, diag, flags = _p1(probe, n)
    N = (n + 1) ** 2
    assert np.array_equal(rp, ref.indptr) and np.array_equal(col, ref.indices)
    assert flags[0] == 1 and flags[1] == 7 and flags[3] == 0
    nslices = (N + 63) // 64
    assert flags[2] == nslices * 448
    # every CSR entry sits at its neighbour offset and its column is stored there
    rows = np.repeat(np.arange(N), np.diff(rp))
    k = (c2s % 448) // 64
    assert np.array_equal(c2s // 448, rows >> 6) and np.array_equal(c2s % 64, rows & 63)
    i, j = rows % (n + 1), rows // (n + 1)
    ci, cj = col % (n + 1), col // (n + 1)
    assert np.array_equal(ci - i, np.take(DI, k)) and np.array_equal(cj - j, np.take(DJ, k))
    assert np.array_equal(scol[c2s], col)
    own = [rp[r] + np.searchsorted(col[rp[r]:rp[r + 1]], r) for r in range(N)]
    assert np.array_equal(col[own], np.arange(N)) and np.array_equal(diag, c2s[own])
    # slots outside the pattern: the row's own column (padding rows: column 0)
    used = np.zeros(flags[2], bool)
    used[c2s] = True
    slot = np.arange(flags[2])
    srow = (slot // 448) * 64 + slot % 64
    pad = ~used
    want = np.where(srow[pad] < N, srow[pad], 0)
    assert np.array_equal(scol[pad], want)
    # rows have 4 (two corners), 3 (the other two), 5 (edges) or 7 entries
    assert sorted(set(np.diff(rp))) == [3, 4, 5, 7]


@pytest.mark.parametrize("n", [8, 16])
def test_elements_match_the_oracle_and_colours_are_conflict_free(probe, n):
    v, ty, cp, np2 = _elements(probe, n)
    m = fem.BoxMesh(n, L10)
    assert np2 == 6 * 2 * n * n and cp[8] == 2 * n * n
    key = lambda t: [tuple(r) for r in t]
    assert sorted(key(v)) == sorted(key(m.tri))
    # type 0 = lower (vertex ids a, a+1, a+n+2), 1 = upper (a, a+n+2, a+n+1)
    a = v[:, 0]
    lo = np.stack([a, a + 1, a + n + 2], 1)
    up = np.stack([a, a + n + 2, a + n + 1], 1)
    assert np.array_equal(v, np.where(ty[:, None] == 0, lo, up))
    for c in range(8):
        vs = v[cp[c]:cp[c + 1]].ravel()
        assert len(np.unique(vs)) == len(vs)


def test_coloured_scatter_reenactment_matches_oracle(probe):
    """Scatter the element matrices of M and K through the slot tables, colour by
    colour, as the device assembly does; read back in CSR order."""
    n, L = 12, L10
    h = L / n
    m = fem.BoxMesh(n, L)
    rp, col, scol, c2s, diag, flags = _p1(probe, n)
    v, ty, cp, _ = _elements(probe, n)
    A = sp.csr_matrix((np.arange(len(col)), col, rp), shape=((n + 1) ** 2,) * 2)
    for which, ref in ((0, fem.p1_mass(m)), (1, fem.p1_stiffness(m))):
        val = np.zeros(flags[2])
        for e in range(len(ty)):
            if ty[e] == 0:
                x1, y1, x2, y2 = h, 0.0, h, h
            else:
                x1, y1, x2, y2 = h, h, 0.0, h
            det = x1 * y2 - x2 * y1
            area = 0.5 * abs(det)
            gx = np.array([0.0, y2 / det, -y1 / det])
            gy = np.array([0.0, -x2 / det, x1 / det])
            gx[0], gy[0] = -gx[1] - gx[2], -gy[1] - gy[2]
            if which == 0:
                loc = area / 12.0 * (np.ones((3, 3)) + np.eye(3))
            else:
                loc = area * (np.outer(gx, gx) + np.outer(gy, gy))
            for p in range(3):
                for q in range(3):
                    val[c2s[A[v[e, p], v[e, q]]]] += loc[p, q]
        got = sp.csr_matrix((val[c2s], col, rp), shape=A.shape)
        assert abs(got - ref).max() < 1e-14 * abs(ref).max()


@pytest.mark.parametrize("nf", [8, 16])
def test_prolongation_and_galerkin_reproduce_the_coarse_forms(probe, nf):
    nc = nf // 2
    fine, coarse = fem.BoxMesh(nf, L10), fem.BoxMesh(nc, L10)
    Nf, Nc = (nf + 1) ** 2, (nc + 1) ** 2
    rp = np.zeros(Nf + 1, np.int32)
    nnz = probe.chns_probe_box_prolongation(nf, _ptr(rp), None, None)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz)
    probe.chns_probe_box_prolongation(nf, _ptr(rp), _ptr(col), _ptr(val))
    P = sp.csr_matrix((val, col, rp), shape=(Nf, Nc))
    # nested P1: interpolating a linear function on the coarse mesh is exact
    xy_f, xy_c = fine.vertex_xy(), coarse.vertex_xy()
    lin = lambda xy: 0.3 * xy[:, 0] - 1.1 * xy[:, 1] + 0.5
    assert np.abs(P @ lin(xy_c) - lin(xy_f)).max() < 1e-13
    assert np.allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0)
    for form in (fem.p1_mass, fem.p1_stiffness):
        Af, Ac = form(fine), form(coarse)
        assert abs(P.T @ Af @ P - Ac).max() < 1e-13 * abs(Ac).max()
        # the library's Galerkin map gives the same coarse values
        got = np.zeros(Ac.nnz)
        assert probe.chns_probe_box_galerkin(nf, _ptr(np.ascontiguousarray(Af.data)), _ptr(got)) == 0
        assert np.abs(got - Ac.data).max() < 1e-13 * abs(Ac).max()


# ---------------------------------------------------------------- Taylor-Hood on the closed square


def _csr_probe(probe, fn, n, *args, nrows):
    rp = np.zeros(nrows + 1, np.int32)
    nnz = fn(n, *args, _ptr(rp), None)
    col = np.zeros(nnz, np.int32)
    fn(n, *args, _ptr(rp), _ptr(col))
    return rp, col


def _pattern(A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A.indptr, A.indices


@pytest.mark.parametrize("n", [8, 12])
def test_box_taylor_hood_tables_match_the_oracle(probe, n):
    probe.chns_probe_box_th_pattern.restype = ct.c_int64
    m = fem.BoxMesh(n, L10)
    N = m.nv
    # element P2 ids: the same six per element (the library orders elements by colour)
    p2 = np.zeros(2 * n * n * 6, np.int32)
    assert probe.chns_probe_box_p2_elements(n, _ptr(p2)) == p2.size
    v, ty, cp, _ = _elements(probe, n)
    lib = {tuple(r[:3]): tuple(r) for r in p2.reshape(-1, 6)}
    assert all(lib[tuple(r[:3])] == tuple(r) for r in m.tri2)
    fixed = np.zeros(4 * N, np.int8)
    assert probe.chns_probe_box_p2_fixed(n, _ptr(fixed)) == 4 * N
    assert np.array_equal(fixed.astype(bool), m.p2_fixed())
    # patterns: the oracle's, plus a lone diagonal on every id of no edge
    used = np.zeros(4 * N, bool)
    used[m.tri2.ravel()] = True
    eye_unused = sp.diags(np.where(used, 0.0, 1.0))
    Mv = fem.p2_mass(m)
    rp, col = _csr_probe(probe, probe.chns_probe_box_th_pattern, n, 0, nrows=4 * N)
    ref = sp.csr_matrix((np.ones(Mv.nnz), Mv.indices, Mv.indptr), shape=Mv.shape) + eye_unused
    ip, ix = _pattern(ref)
    assert np.array_equal(rp, ip) and np.array_equal(col, ix)
    B = fem.divergence_matrix(m)
    rp, col = _csr_probe(probe, probe.chns_probe_box_th_pattern, n, 1, nrows=N)
    ib = sp.csr_matrix((np.ones(B.nnz), B.indices, B.indptr), shape=B.shape)
    ip, ix = _pattern(ib)
    assert np.array_equal(rp, ip) and np.array_equal(col, ix)
    # velocity rows couple to both components on the P2 pattern and to pressure
    vv = sp.bmat([[Mv, Mv], [Mv, Mv]])
    A = sp.bmat([[vv, B.T], [B, None]]).tocsr()
    ones = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    ones = ones + sp.diags(np.concatenate([np.where(used, 0.0, 1.0)] * 2 + [np.zeros(N)]))
    rp, col = _csr_probe(probe, probe.chns_probe_box_th_pattern, n, 2, nrows=9 * N)
    ip, ix = _pattern(ones)
    assert np.array_equal(rp, ip) and np.array_equal(col, ix)


def test_box_p1_to_p2_transfer(probe):
    """The P1 -> P2 transfer of the velocity hierarchy: linear fields exact at
    every P2 id off the no-slip set, no row on it."""
    n = 10
    m = fem.BoxMesh(n, L10)
    N = m.nv
    rp = np.zeros(4 * N + 1, np.int32)
    nnz = probe.chns_probe_box_p2_transfer(n, _ptr(rp), None, None)
    col, val = np.zeros(nnz, np.int32), np.zeros(nnz)
    probe.chns_probe_box_p2_transfer(n, _ptr(rp), _ptr(col), _ptr(val))
    P = sp.csr_matrix((val, col, rp), shape=(4 * N, N))
    fixed = m.p2_fixed()
    assert np.all(np.diff(rp)[fixed] == 0)
    lin = lambda xy: 0.7 * xy[:, 0] - 0.2 * xy[:, 1] + 1.0
    got = P @ lin(m.vertex_xy())
    assert np.abs(got[~fixed] - lin(m.p2_xy())[~fixed]).max() < 1e-12


@pytest.mark.parametrize("n", [8, 16, 66])
def test_box_transfer_sell_columns_stay_in_range(probe, n):
    """The P1 -> P2 transfer of the closed square ends with rows of no entry
    (ids of no edge); their SELL padding must still name a valid column (the
    kernels read x at every stored column)."""
    assert probe.chns_probe_box_p2_transfer_sell_bad(n) == 0
