"""Pins of the oracle on the periodic cube (Kuhn tetrahedra, P1): the paper's
three-dimensional discretisation (section "Numerical results": uniform
tetrahedral meshes, linear Lagrange elements) for the binary models.

Pinned against facts fixed independently of the assembly: the mesh's volumes
and edge set, the known identity of the Kuhn mesh's P1 stiffness matrix with h
times the 7-point finite-difference Laplacian, the exact mass of constants, a
manufactured Helmholtz problem at second order, the mesh's symmetries (axis
permutations and the point reflection), conservation, constant states and the
energy decay of small steps."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem3d, potential as pot, step as S
from oracle.systems import Params


def _ids(n, i, j, k):
    return (i % n) + n * (j % n) + n * n * (k % n)


def test_mesh_volumes_edges_and_orientation():
    n = 5
    m = fem3d.Mesh3(n)
    assert m.ne == 6 * n ** 3
    assert np.allclose(m.vol, m.h ** 3 / 6) and abs(m.vol.sum() - 1.0) < 1e-13
    edges = set()
    for t in m.tet:
        for a in range(4):
            for b in range(a + 1, 4):
                edges.add((min(t[a], t[b]), max(t[a], t[b])))
    assert len(edges) == 7 * n ** 3  # seven edge directions per vertex
    # every tetrahedron's vertices sit at its coordinates (mod the period)
    xyz = m.vertex_xyz()
    assert np.allclose(xyz[m.tet], m.xyz % 1.0)


def test_stiffness_is_h_times_the_seven_point_laplacian():
    n = 6
    m = fem3d.Mesh3(n)
    K = fem3d.p1_stiffness(m).tocsr()
    N = n ** 3
    k, j, i = np.unravel_index(np.arange(N), (n, n, n))
    rows = np.repeat(np.arange(N), 7)
    cols = np.stack([np.arange(N), _ids(n, i + 1, j, k), _ids(n, i - 1, j, k), _ids(n, i, j + 1, k),
                     _ids(n, i, j - 1, k), _ids(n, i, j, k + 1), _ids(n, i, j, k - 1)], 1).ravel()
    vals = np.tile([6.0, -1, -1, -1, -1, -1, -1], N) * m.h
    ref = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    assert abs(K - ref).max() < 1e-14
    assert set(np.diff(K.indptr)) == {15}  # the pattern keeps the 14 neighbours


def test_mass_matrix_exact_on_constants_and_symmetric():
    m = fem3d.Mesh3(4, 2.0)
    M = fem3d.p1_mass(m)
    one = np.ones(m.nv)
    assert np.allclose(M @ one, m.h ** 3) and abs(one @ (M @ one) - 8.0) < 1e-13
    assert abs(M - M.T).max() == 0.0
    assert np.linalg.eigvalsh(M.toarray()).min() > 0


def test_helmholtz_converges_at_second_order():
    """(M + K) u_h = (f, phi_i) for -lap u + u = f, u = cos 2 pi x cos 2 pi y cos 2 pi z:
    the L^2 error falls at second order (1.82 then 1.95 on 12, 24, 48 cells;
    the coarsest mesh resolves the mode with 12 points)."""
    import scipy.sparse.linalg as spla
    tp = 2 * np.pi
    u = lambda x, y, z: np.cos(tp * x) * np.cos(tp * y) * np.cos(tp * z)
    f = lambda x, y, z: (1 + 3 * tp ** 2) * u(x, y, z)
    errs = []
    for n in (12, 24, 48):
        m = fem3d.Mesh3(n)
        M = fem3d.p1_mass(m)
        uh, info = spla.cg(M + fem3d.p1_stiffness(m), fem3d.p1_load(m, f), rtol=1e-13, maxiter=5000)
        assert info == 0
        xyz = m.vertex_xyz()
        e = uh - u(xyz[:, 0], xyz[:, 1], xyz[:, 2])
        errs.append(np.sqrt(e @ (M @ e)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[0] > 1.75 and rates[1] > 1.9 and rates[1] > rates[0], (errs, rates)


PC = dict(eps=0.05, tau=1e-4, mobility=1.0, evap_rate=0.5)


def _state(n, model, seed, mean=0.5, amp=0.01):
    g = np.random.default_rng(seed)
    N = n ** 3
    f = dict(phi=[mean + amp * g.uniform(-1, 1, N)], Phi_v=None, vel=None, p=None)
    if model == "ch_ac":
        z = fem3d.Mesh3(n).vertex_xyz()[:, 2]
        f["Phi_v"] = np.sin(np.pi * z) ** 2
    return f


@pytest.mark.parametrize("model", ["ch", "ch_ac"])
def test_step_conserves_mass_and_dense_equals_sparse(model):
    n = 6
    ops, prm = S.Operators3D(n), Params(**PC)
    st = S.initial_state(ops, prm, model, _state(n, model, 1))
    a = S.step(ops, prm, model, st, "dense")
    b = S.step(ops, prm, model, st, "splu")
    assert np.abs(a["phi"][0] - b["phi"][0]).max() < 1e-12
    assert abs(S.mass(ops, b["phi"][0]) - S.mass(ops, st["phi"][0])) < 1e-14
    with pytest.raises(ValueError):
        S.step(ops, prm, model, st, "fft")


def test_constant_state_and_reaction():
    n = 4
    ops, prm = S.Operators3D(n), Params(**PC)
    c, cv = 0.3, 0.7
    st = S.initial_state(ops, prm, "ch_ac", dict(phi=[np.full(ops.N, c)], Phi_v=np.full(ops.N, cv)))
    out = S.step(ops, prm, "ch_ac", st)
    assert np.abs(out["phi"][0] - c).max() < 1e-13
    assert np.abs(out["mu"][0] - pot.dfdphi_bin(c, cv)).max() < 1e-12
    assert np.abs(out["Phi_v"] - (cv - prm.tau * prm.gamma_v * pot.dfdPhi_bin(c, cv))).max() < 1e-13


@pytest.mark.parametrize("which", ["xy", "yz", "reflect"])
def test_step_commutes_with_the_mesh_symmetries(which):
    """The Kuhn mesh of the periodic cube is invariant under permutations of
    the axes and under the point reflection x -> -x; so is the step."""
    n = 6
    ops, prm = S.Operators3D(n), Params(**PC)
    g = np.random.default_rng(3)
    phi = 0.5 + 0.1 * g.uniform(-1, 1, ops.N)
    Phi = 0.5 + 0.3 * g.uniform(-1, 1, ops.N)
    k, j, i = np.unravel_index(np.arange(ops.N), (n, n, n))
    P = {"xy": _ids(n, j, i, k), "yz": _ids(n, i, k, j), "reflect": _ids(n, -i, -j, -k)}[which]
    a = S.step(ops, prm, "ch_ac", S.initial_state(ops, prm, "ch_ac", dict(phi=[phi], Phi_v=Phi)))
    b = S.step(ops, prm, "ch_ac", S.initial_state(ops, prm, "ch_ac", dict(phi=[phi[P]], Phi_v=Phi[P])))
    for x, y in ((a["phi"][0], b["phi"][0]), (a["mu"][0], b["mu"][0]), (a["Phi_v"], b["Phi_v"])):
        assert np.abs(x[P] - y).max() < 1e-11 * np.abs(x).max()


def test_small_steps_decrease_the_energy():
    """From phi = 0.3 +- 0.1 (off the double well's symmetry point, where the
    lumped-mass energy's change is set by the mass lumping, not by the flow)."""
    n = 6
    ops, prm = S.Operators3D(n), Params(**dict(PC, tau=1e-6))
    st = S.initial_state(ops, prm, "ch", _state(n, "ch", 4, mean=0.3, amp=0.1))
    E = [S.energy_ch(ops, prm, st["phi"][0])]
    for _ in range(3):
        out = S.step(ops, prm, "ch", st)
        st = dict(st, phi=out["phi"], mu=out["mu"])
        E.append(S.energy_ch(ops, prm, st["phi"][0]))
    assert all(E[i + 1] < E[i] for i in range(3)), E


@pytest.mark.parametrize("nf", [8, 12])
def test_cube_prolongation_is_nested(nf):
    """P^T A_h P equals the coarse mesh's own form (the Kuhn meshes are nested,
    so the coarse P1 space is a subspace of the fine one), and P copies the
    coarse vertices."""
    from oracle import multigrid as mg
    P = mg.prolongation_cube(nf)
    nc = nf // 2
    assert P.shape == (nf ** 3, nc ** 3) and np.allclose(P @ np.ones(nc ** 3), 1.0)
    g = np.random.default_rng(1).standard_normal(nc ** 3)
    kk, jj, ii = np.meshgrid(np.arange(nc), np.arange(nc), np.arange(nc), indexing="ij")
    assert np.array_equal((P @ g)[_ids(nf, 2 * ii, 2 * jj, 2 * kk).ravel()], g)
    for form in (fem3d.p1_mass, fem3d.p1_stiffness):
        ref = form(fem3d.Mesh3(nc, 2.0))
        assert abs(P.T @ form(fem3d.Mesh3(nf, 2.0)) @ P - ref).max() <= 1e-14 * abs(ref).max()


def test_cube_smoother_bounds_hold():
    """The spectral facts the cube's cycle rests on: D^{-1} M in [0.5, 2.5],
    D^{-1} K in [0, 2], so D^{-1}(a M + b K) stays below LMAX_CUBE and above
    0.5 / (1 + 15 b / (a h^2))."""
    from oracle import multigrid as mg
    n = 6
    m = fem3d.Mesh3(n, 1.5)
    M, K = fem3d.p1_mass(m).toarray(), fem3d.p1_stiffness(m).toarray()
    ev = lambda A: np.linalg.eigvals(A / A.diagonal()[:, None]).real
    em, ek = ev(M), ev(K)
    assert em.min() > 0.5 - 1e-12 and em.max() < 2.5 + 1e-12 and abs(em.max() - 2.5) < 1e-9
    assert ek.min() > -1e-12 and ek.max() < 2.0 + 1e-12
    for a, b in ((1.0, 0.0), (1.0, 1e-3), (0.3, 0.05), (1.0, 10.0)):
        e = ev(a * M + b * K)
        assert e.max() < mg.LMAX_CUBE
        assert e.min() >= 0.5 / (1.0 + mg.rho(a, b, n, 1.5, cube=True)) - 1e-12, (a, b)


@pytest.mark.parametrize("n", [8, 16])
def test_cube_cycle_contracts(n):
    """One V(2, 1) cycle on the matching factor tau g K + sqrt(tau g / beta) M
    contracts the error by a mesh-independent factor."""
    from oracle import multigrid as mg
    prm = Params(**PC)
    t, g, b = prm.tau, prm.gamma, prm.beta
    m = fem3d.Mesh3(n)
    X = (t * g * fem3d.p1_stiffness(m) + np.sqrt(t * g / b) * fem3d.p1_mass(m)).tocsr()
    H = mg.Hierarchy(X, n, a=np.sqrt(t * g / b), b=t * g, cube_length=1.0)
    assert len(H.A) >= 2  # the operator is cut below the fine level
    e = np.random.default_rng(2).standard_normal(n ** 3)
    for _ in range(4):
        e = e - mg.vcycle(H, X @ e, pre=2, post=1, coarse=12)
    e1 = e - mg.vcycle(H, X @ e, pre=2, post=1, coarse=12)
    assert np.linalg.norm(e1) < 0.35 * np.linalg.norm(e)
