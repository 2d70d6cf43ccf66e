"""Pins of the oracle on the closed cube [0, L]^3 (Kuhn tetrahedra, (n+1)^3
vertices, no identification): the paper's three-dimensional domain with the
natural (no-flux) conditions of the phase and vapour fields and the
evaporation flux through the top face (eq. (bc)).

Pinned against facts fixed independently of the assembly: volumes and counts,
exact forms on linear fields, a manufactured Neumann problem at second order,
the top-face load against exact face integrals of linear functions, nested
prolongation, the element bounds of the smoother, and step invariants
(conservation, constant states, symmetries, the flux's linearity, energy
decay)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem3d, multigrid as mg, potential as pot, step as S
from oracle.systems import Params

L3 = 2.0
PC = dict(eps=0.3, tau=1e-3, mobility=1.0, evap_rate=0.5)


def _ids(m, i, j, k):
    return i + m * j + m * m * k


def test_mesh_counts_volumes_and_linear_forms():
    n = 4
    m = fem3d.Mesh3(n, L3, box=True)
    assert m.nv == (n + 1) ** 3 and m.ne == 6 * n ** 3
    assert abs(m.vol.sum() - L3 ** 3) < 1e-12 and np.allclose(m.vol, m.h ** 3 / 6)
    assert np.unique(m.tet).size == m.nv
    xyz = m.vertex_xyz()
    assert np.allclose(xyz[m.tet], m.xyz)
    M, K = fem3d.p1_mass(m), fem3d.p1_stiffness(m)
    one = np.ones(m.nv)
    assert np.abs(K @ one).max() < 1e-13 and abs(one @ (M @ one) - L3 ** 3) < 1e-12
    a = np.array([0.3, -1.1, 0.7])
    u = xyz @ a + 0.4
    assert abs(u @ (K @ u) - (a @ a) * L3 ** 3) < 1e-11
    # int u^2 for linear u, exact: the P1 mass integrates products of linears exactly
    exact = (0.4 ** 2) * L3 ** 3 + 2 * 0.4 * a.sum() * L3 ** 4 / 2 + \
        sum(a[i] * a[j] * (L3 ** 5 / 3 if i == j else L3 ** 5 / 4) for i in range(3) for j in range(3))
    assert abs(u @ (M @ u) - exact) < 1e-11 * exact


def test_top_face_load_is_exact_on_linear_functions():
    n = 6
    m = fem3d.Mesh3(n, L3, box=True)
    b = fem3d.top_face_load(m)
    xyz = m.vertex_xyz()
    assert np.all(b[~np.isclose(xyz[:, 2], L3)] == 0.0)
    assert abs(b.sum() - L3 ** 2) < 1e-13
    g = 1.0 + 0.5 * xyz[:, 0] - 0.25 * xyz[:, 1]
    assert abs(b @ g - (L3 ** 2 + 0.5 * L3 ** 3 / 2 - 0.25 * L3 ** 3 / 2)) < 1e-12
    with pytest.raises(ValueError):
        fem3d.top_face_load(fem3d.Mesh3(n, L3))


def test_neumann_helmholtz_converges_at_second_order():
    """(M + K) u_h = (f, phi_i) for -lap u + u = f with the natural condition,
    u = cos(pi x/L) cos(pi y/L) cos(pi z/L) (zero normal derivative on every
    face): L^2 error at second order."""
    k = np.pi / L3
    u = lambda x, y, z: np.cos(k * x) * np.cos(k * y) * np.cos(k * z)
    f = lambda x, y, z: (1 + 3 * k * k) * u(x, y, z)
    errs = []
    for n in (6, 12, 24):
        m = fem3d.Mesh3(n, L3, box=True)
        M = fem3d.p1_mass(m)
        uh, info = spla.cg(M + fem3d.p1_stiffness(m), fem3d.p1_load(m, f), rtol=1e-13, maxiter=5000)
        assert info == 0
        xyz = m.vertex_xyz()
        e = uh - u(xyz[:, 0], xyz[:, 1], xyz[:, 2])
        errs.append(np.sqrt(e @ (M @ e)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 1.8, (errs, rates)


@pytest.mark.parametrize("nf", [4, 8])
def test_box_prolongation_is_nested(nf):
    P = mg.prolongation_cube_box(nf)
    nc = nf // 2
    assert P.shape == ((nf + 1) ** 3, (nc + 1) ** 3) and np.allclose(P @ np.ones(P.shape[1]), 1.0)
    # linear fields are reproduced exactly
    xc = fem3d.Mesh3(nc, L3, box=True).vertex_xyz()
    xf = fem3d.Mesh3(nf, L3, box=True).vertex_xyz()
    a = np.array([0.2, 0.5, -0.9])
    assert np.abs(P @ (xc @ a) - xf @ a).max() < 1e-13
    for form in (fem3d.p1_mass, fem3d.p1_stiffness):
        ref = form(fem3d.Mesh3(nc, L3, box=True))
        got = P.T @ form(fem3d.Mesh3(nf, L3, box=True)) @ P
        assert abs(got - ref).max() <= 1e-14 * abs(ref).max()


def test_smoother_bounds_hold_on_the_closed_cube():
    """The element bounds of the cube's cycle hold with the walls: D^{-1} M in
    [0.5, 2.5], D^{-1} K in [0, 2]."""
    m = fem3d.Mesh3(4, L3, box=True)
    M, K = fem3d.p1_mass(m).toarray(), fem3d.p1_stiffness(m).toarray()
    ev = lambda A: np.linalg.eigvals(A / A.diagonal()[:, None]).real
    em, ek = ev(M), ev(K)
    assert em.min() > 0.5 - 1e-12 and em.max() < 2.5 + 1e-12
    assert ek.min() > -1e-12 and ek.max() < 2.0 + 1e-12
    assert ek.max() < mg.LMAX_CUBE and em.max() < mg.LMAX_CUBE


def _state(n, model, seed, mean=0.4, amp=0.05):
    m = fem3d.Mesh3(n, L3, box=True)
    g = np.random.default_rng(seed)
    f = dict(phi=[mean + amp * g.uniform(-1, 1, m.nv)], Phi_v=None, vel=None, p=None)
    if model == "ch_ac":
        z = m.vertex_xyz()[:, 2]
        f["Phi_v"] = np.clip(z / L3, 0.0, 1.0) ** 2
    return f


@pytest.mark.parametrize("model", ["ch", "ch_ac"])
def test_step_conserves_mass_and_dense_equals_sparse(model):
    n = 4
    ops, prm = S.Operators3D(n, L3, box=True), Params(**PC)
    st = S.initial_state(ops, prm, model, _state(n, model, 1))
    a = S.step(ops, prm, model, st, "dense")
    b = S.step(ops, prm, model, st, "splu")
    assert np.abs(a["phi"][0] - b["phi"][0]).max() < 1e-12
    assert abs(S.mass(ops, b["phi"][0]) - S.mass(ops, st["phi"][0])) < 1e-13 * abs(S.mass(ops, st["phi"][0]))


def test_constant_state_and_reaction():
    n = 4
    ops, prm = S.Operators3D(n, L3, box=True), Params(**PC)
    c, cv = 0.3, 0.7
    st = S.initial_state(ops, prm, "ch_ac", dict(phi=[np.full(ops.N, c)], Phi_v=np.full(ops.N, cv)))
    out = S.step(ops, prm, "ch_ac", st)
    assert np.abs(out["phi"][0] - c).max() < 1e-13
    assert np.abs(out["mu"][0] - pot.dfdphi_bin(c, cv)).max() < 1e-12
    assert np.abs(out["Phi_v"] - (cv - prm.tau * prm.gamma_v * pot.dfdPhi_bin(c, cv))).max() < 1e-13


@pytest.mark.parametrize("which", ["xy", "reflect"])
def test_step_commutes_with_the_mesh_symmetries(which):
    """The closed cube's Kuhn mesh is invariant under permutations of the
    axes and the point reflection through the centre; so is the step without
    the flux (whose face breaks both)."""
    n = 4
    m1 = n + 1
    ops, prm = S.Operators3D(n, L3, box=True), Params(**PC)
    g = np.random.default_rng(3)
    phi = 0.5 + 0.1 * g.uniform(-1, 1, ops.N)
    Phi = 0.5 + 0.3 * g.uniform(-1, 1, ops.N)
    k, j, i = np.unravel_index(np.arange(ops.N), (m1, m1, m1))
    P = {"xy": _ids(m1, j, i, k), "reflect": _ids(m1, n - i, n - j, n - k)}[which]
    a = S.step(ops, prm, "ch_ac", S.initial_state(ops, prm, "ch_ac", dict(phi=[phi], Phi_v=Phi)))
    b = S.step(ops, prm, "ch_ac", S.initial_state(ops, prm, "ch_ac", dict(phi=[phi[P]], Phi_v=Phi[P])))
    for x, y in ((a["phi"][0], b["phi"][0]), (a["mu"][0], b["mu"][0]), (a["Phi_v"], b["Phi_v"])):
        assert np.abs(x[P] - y).max() < 1e-11 * np.abs(x).max()


def test_top_face_flux_is_linear_and_keeps_the_phase_mass():
    """The flux loads the second CH equation with j_out int_top phi_i dS:
    nothing at phi_ref = phi_inf, a response linear in the rate, the phase
    mass unchanged (1^T K = 0), and the phase drawn towards the face for
    j_out > 0 (mu lowered there)."""
    n = 4
    ops = S.Operators3D(n, L3, box=True)
    st0 = S.initial_state(ops, Params(**PC), "ch", _state(n, "ch", 2))
    ref_id = n // 2 + (n + 1) * (n // 2) + (n + 1) ** 2 * n
    base = S.step(ops, Params(**PC), "ch", st0)
    same = S.step(ops, Params(**PC, top_flux=3.0, flux_inf=st0["phi"][0][ref_id]), "ch", st0)
    assert np.abs(same["phi"][0] - base["phi"][0]).max() < 1e-14
    d1 = S.step(ops, Params(**PC, top_flux=1.0, flux_inf=0.0), "ch", st0)["phi"][0] - base["phi"][0]
    d2 = S.step(ops, Params(**PC, top_flux=2.0, flux_inf=0.0), "ch", st0)["phi"][0] - base["phi"][0]
    assert np.abs(d2 - 2 * d1).max() < 1e-9 * np.abs(d2).max() and np.abs(d1).max() > 0
    assert abs(S.mass(ops, base["phi"][0] + d1) - S.mass(ops, st0["phi"][0])) < 1e-13 * abs(S.mass(ops, st0["phi"][0]))
    top = np.isclose(ops.mesh.vertex_xyz()[:, 2], L3)
    assert d1[top].mean() > 0 > d1[~top].mean()


def test_small_steps_decrease_the_energy():
    n = 4
    ops, prm = S.Operators3D(n, L3, box=True), Params(**dict(PC, tau=1e-6))
    st = S.initial_state(ops, prm, "ch", _state(n, "ch", 4, mean=0.3, amp=0.1))
    E = [S.energy_ch(ops, prm, st["phi"][0])]
    for _ in range(3):
        out = S.step(ops, prm, "ch", st)
        st = dict(st, phi=out["phi"], mu=out["mu"])
        E.append(S.energy_ch(ops, prm, st["phi"][0]))
    assert all(E[i + 1] < E[i] for i in range(3)), E
