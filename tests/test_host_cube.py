"""CPU checks of the library's host tables on the cube (Kuhn tetrahedra):
periodic (n^3 vertices i + n j + n^2 k) and closed ((n+1)^3 vertices, no
identification).  The tetrahedra and their 48-colour order against the
oracle's mesh, the 15-point P1 pattern and its SELL layout (every stored
column and slot in range; on the closed cube a neighbour outside it stored as
the row's own column), the element slot tables by a re-enactment of the
coloured scatter with the oracle's element matrices, the nested prolongation
with its Galerkin map against the oracle's coarse-mesh forms (P^T A_h P = A_2h
holds exactly for nested P1 spaces), and the closed cube's top-face weights
against the oracle's face integrals."""
import ctypes as ct
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem3d

PROBE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2501_11767_amd", "libchns_hostprobe.so")


@pytest.fixture(scope="module")
def probe():
    if not os.path.exists(PROBE):
        pytest.skip("host probe library not built")
    L = ct.CDLL(PROBE)
    L.chns_probe_cube_p1.restype = ct.c_int64
    return L


def _ptr(a):
    return a.ctypes.data_as(ct.c_void_p)


def _tets(probe, n, box=0):
    ne = 6 * n ** 3
    v = np.zeros(ne * 4, np.int32)
    ty = np.zeros(ne, np.int32)
    cp = np.zeros(49, np.int32)
    assert probe.chns_probe_cube_tets(n, box, _ptr(v), _ptr(ty), _ptr(cp)) == ne
    return v.reshape(ne, 4), ty, cp


def _p1(probe, n, box=0):
    N = (n + box) ** 3
    nnz = probe.chns_probe_cube_p1(n, box, None, None, None, None, None, None, None)
    flags = np.zeros(4, np.int32)
    rp = np.zeros(N + 1, np.int32)
    col = np.zeros(nnz, np.int32)
    probe.chns_probe_cube_p1(n, box, _ptr(rp), _ptr(col), None, None, None, _ptr(flags), None)
    scol = np.zeros(flags[2], np.int32)
    c2s = np.zeros(nnz, np.int32)
    diag = np.zeros(N, np.int32)
    es = np.zeros(6 * n ** 3 * 16, np.int32)
    probe.chns_probe_cube_p1(n, box, None, None, _ptr(scol), _ptr(c2s), _ptr(diag), None, _ptr(es))
    return rp, col, scol, c2s, diag, flags, es.reshape(-1, 16)


@pytest.mark.parametrize("n,box", [(4, 0), (6, 0), (8, 0), (4, 1), (6, 1)])
def test_tetrahedra_match_the_oracle_and_colours_are_independent(probe, n, box):
    v, ty, cp = _tets(probe, n, box)
    m = fem3d.Mesh3(n, box=bool(box))
    mine = sorted(map(tuple, np.concatenate([v, ty[:, None]], 1).tolist()))
    ref = sorted(map(tuple, np.concatenate([m.tet, m.type[:, None]], 1).tolist()))
    assert mine == ref  # same vertex order within each tetrahedron, same types
    assert cp[0] == 0 and cp[48] == v.shape[0] and np.all(np.diff(cp) == n ** 3 // 8)
    for c in range(48):
        block = v[cp[c]:cp[c + 1]].ravel()
        assert np.unique(block).size == block.size, c  # no vertex twice in a colour
        assert np.all(ty[cp[c]:cp[c + 1]] == c >> 3)


@pytest.mark.parametrize("n,box", [(4, 0), (6, 0), (8, 0), (4, 1), (6, 1)])
def test_pattern_and_sell_layout(probe, n, box):
    m = n + box
    N = m ** 3
    rp, col, scol, c2s, diag, flags, es = _p1(probe, n, box)
    K = fem3d.p1_stiffness(fem3d.Mesh3(n, box=bool(box))).tocsr()
    assert np.array_equal(rp, K.indptr) and np.array_equal(col, K.indices)
    assert flags[0] == 1 and flags[1] == 15 and flags[2] == ((N + 63) // 64) * 64 * 15
    assert scol.min() >= 0 and scol.max() < N  # padding lanes name column 0
    assert np.unique(c2s).size == c2s.size and c2s.min() >= 0 and c2s.max() < flags[2]
    # SELL slot q of row r holds lane r % 64 of slice r // 64
    r = np.repeat(np.arange(N), np.diff(rp))
    assert np.all((c2s % 64) == (r % 64)) and np.all(c2s // (64 * 15) == r // 64)
    assert np.array_equal(scol[c2s], col)
    assert np.array_equal(scol[diag], np.arange(N))
    assert es.min() >= 0 and es.max() < flags[2]
    # entry k of row (i, j, l) is the fixed neighbour the kernels compute (the
    # vertex, then -d and +d for each edge direction in turn); on the closed
    # cube a neighbour outside it is the row itself and the columns are stored
    assert flags[3] == (0 if box else n)
    dirs = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]
    offs = [(0, 0, 0)] + [tuple(sg * np.array(d)) for d in dirs for sg in (-1, 1)]
    l, j, i = np.unravel_index(np.arange(N), (m, m, m))
    for k, (a, b, c) in enumerate(offs):
        if box:
            inside = (i + a >= 0) & (i + a < m) & (j + b >= 0) & (j + b < m) & (l + c >= 0) & (l + c < m)
            want = np.where(inside, (i + a) + m * (j + b) + m * m * (l + c), np.arange(N))
        else:
            want = (i + a) % n + n * ((j + b) % n) + n * n * ((l + c) % n)
        slots = (np.arange(N) // 64) * 64 * 15 + k * 64 + np.arange(N) % 64
        assert np.array_equal(scol[slots], want), k


@pytest.mark.parametrize("box", [0, 1])
def test_coloured_scatter_reenacted_with_the_oracle_element_matrices(probe, box):
    """The library's slot table (eslot) scatters each tetrahedron's 4 x 4 block:
    with the oracle's element matrices the SELL values read back as the
    oracle's assembled mass and stiffness matrices."""
    n = 6
    v, ty, cp = _tets(probe, n, box)
    rp, col, scol, c2s, diag, flags, es = _p1(probe, n, box)
    m = fem3d.Mesh3(n, box=bool(box))
    key = {t: i for i, t in enumerate(map(tuple, m.tet.tolist()))}
    order = np.array([key[t] for t in map(tuple, v.tolist())])  # library element -> oracle element
    Me = np.broadcast_to(m.vol[:, None, None] * (np.ones((4, 4)) + np.eye(4)) / 20.0, (m.ne, 4, 4))
    Ke = np.einsum("e,ead,ebd->eab", m.vol, m.grad, m.grad)
    for Ae, ref in ((Me, fem3d.p1_mass(m)), (Ke, fem3d.p1_stiffness(m))):
        val = np.zeros(flags[2])
        for c in range(48):
            e = np.arange(cp[c], cp[c + 1])
            np.add.at(val, es[e].ravel(), Ae[order[e]].reshape(-1))
        got = sp.csr_matrix((val[c2s], col, rp), shape=(m.nv,) * 2)
        assert abs(got - ref).max() <= 1e-15 * abs(ref).max()
        pad = np.ones(flags[2], bool)
        pad[c2s] = False
        assert np.all(val[pad] == 0.0)


def _prolongation(probe, nf, box=0):
    nnz = probe.chns_probe_cube_prolongation(nf, box, None, None, None)
    rp = np.zeros((nf + box) ** 3 + 1, np.int32)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz)
    probe.chns_probe_cube_prolongation(nf, box, _ptr(rp), _ptr(col), _ptr(val))
    return sp.csr_matrix((val, col, rp), shape=((nf + box) ** 3, (nf // 2 + box) ** 3))


@pytest.mark.parametrize("nf", [8, 12])
def test_prolongation_is_the_nested_interpolation(probe, nf):
    P = _prolongation(probe, nf, 0)
    assert np.allclose(P @ np.ones(P.shape[1]), 1.0)
    # a coarse P1 function sampled at the fine vertices: fine vertex (2I, 2J, 2K)
    # is coarse vertex (I, J, K)
    nc = nf // 2
    g = np.random.default_rng(0).standard_normal(nc ** 3)
    f = P @ g
    kk, jj, ii = np.meshgrid(np.arange(nc), np.arange(nc), np.arange(nc), indexing="ij")
    fid = (2 * ii + nf * 2 * jj + nf * nf * 2 * kk).ravel()
    assert np.array_equal(f[fid], g)
    for Mf, Mc in ((fem3d.p1_mass, fem3d.p1_mass), (fem3d.p1_stiffness, fem3d.p1_stiffness)):
        A = Mf(fem3d.Mesh3(nf, 2.0))
        ref = Mc(fem3d.Mesh3(nc, 2.0))
        assert abs(P.T @ A @ P - ref).max() <= 1e-14 * abs(ref).max()


@pytest.mark.parametrize("nf", [8, 12])
def test_galerkin_map_gives_the_coarse_forms(probe, nf):
    for form in (fem3d.p1_mass, fem3d.p1_stiffness):
        A = form(fem3d.Mesh3(nf, 3.0)).tocsr()
        A.sort_indices()
        ref = form(fem3d.Mesh3(nf // 2, 3.0)).tocsr()
        ref.sort_indices()
        out = np.zeros(ref.nnz)
        assert probe.chns_probe_cube_galerkin(nf, 0, _ptr(np.ascontiguousarray(A.data)), _ptr(out)) == 0
        assert np.abs(out - ref.data).max() <= 1e-14 * np.abs(ref.data).max()


@pytest.mark.parametrize("nf", [4, 8])
def test_closed_cube_prolongation_and_galerkin(probe, nf):
    """The closed cube: the prolongation equals the oracle's box
    interpolation, and the Galerkin map gives the coarse forms."""
    from oracle import multigrid as mg
    P = _prolongation(probe, nf, 1)
    assert abs(P - mg.prolongation_cube_box(nf)).max() == 0.0
    for form in (fem3d.p1_mass, fem3d.p1_stiffness):
        A = form(fem3d.Mesh3(nf, 3.0, box=True)).tocsr()
        A.sort_indices()
        ref = form(fem3d.Mesh3(nf // 2, 3.0, box=True)).tocsr()
        ref.sort_indices()
        out = np.zeros(ref.nnz)
        assert probe.chns_probe_cube_galerkin(nf, 1, _ptr(np.ascontiguousarray(A.data)), _ptr(out)) == 0
        assert np.abs(out - ref.data).max() <= 1e-14 * np.abs(ref.data).max()


@pytest.mark.parametrize("n", [4, 6])
def test_closed_cube_top_face_weights_match_the_oracle(probe, n):
    L = 2.5
    w = np.zeros((n + 1) ** 2)
    assert probe.chns_probe_cube_top_weights(n, ct.c_double(L / n), _ptr(w)) == (n + 1) ** 2
    ref = fem3d.top_face_load(fem3d.Mesh3(n, L, box=True))[n * (n + 1) ** 2:]
    assert np.abs(w - ref).max() <= 1e-15 * L * L and abs(w.sum() - L * L) < 1e-13
