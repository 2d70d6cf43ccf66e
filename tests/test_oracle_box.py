"""Pins of the oracle on the paper's closed domain: the square [0, L]^2 with
no-flux boundary conditions (eq. (bc) for the phase fields, the chemical
potentials and the vapour field; section "Numerical results" for the 10 x 10
square), where the natural boundary conditions come with P1 forms assembled
without boundary terms.

Pinned against what mathematics fixes independently of the assembly: exact
integrals of linear functions, the boundary flux that Green's formula leaves in
K u for a linear u, the second-order convergence of a Neumann problem with a
known solution, conservation of the phase mass, constant states, the mesh's
symmetries and the energy decay of small steps."""
import numpy as np
import pytest

from oracle import fem, potential as pot, solvers, step as S
from oracle.systems import Params
from paper_2501_11767_amd import inputs

L10 = 10.0


def test_box_mesh_numbering_and_geometry():
    n, L = 6, 2.5
    m = fem.BoxMesh(n, L)
    assert m.nv == (n + 1) ** 2 and m.ne == 2 * n * n
    assert np.allclose(m.area, 0.5 * (L / n) ** 2) and abs(m.area.sum() - L * L) < 1e-13
    xy = m.vertex_xy()
    assert np.array_equal(xy, inputs.box_vertex_coords(n, L))
    assert np.allclose(m.xy, xy[m.tri])  # element coordinates are those of its vertices
    # every interior edge is shared by two triangles, every boundary edge by one
    edges = np.sort(np.concatenate([m.tri[:, [0, 1]], m.tri[:, [1, 2]], m.tri[:, [0, 2]]]), axis=1)
    _, cnt = np.unique(edges, axis=0, return_counts=True)
    assert (cnt == 1).sum() == 4 * n and set(cnt) == {1, 2}


def _linear(m, a, b, c):
    xy = m.vertex_xy()
    return a * xy[:, 0] + b * xy[:, 1] + c


@pytest.mark.parametrize("n,L", [(4, 1.0), (8, L10)])
def test_p1_forms_are_exact_on_linear_functions(n, L):
    m = fem.BoxMesh(n, L)
    M, K = fem.p1_mass(m), fem.p1_stiffness(m)
    a, b, c = 0.7, -1.3, 0.4
    u = _linear(m, a, b, c)
    # int |grad u|^2 and int u^2 over the square (P1 holds linear functions exactly)
    assert abs(u @ (K @ u) - (a * a + b * b) * L * L) < 1e-12 * L * L
    ref = (a * a + b * b) * L ** 4 / 3 + c * c * L * L + a * b * L ** 4 / 2 + (a + b) * c * L ** 3
    assert abs(u @ (M @ u) - ref) < 1e-12 * abs(ref)
    assert np.abs(K @ np.ones(m.nv)).max() < 1e-13
    assert abs(np.ones(m.nv) @ (M @ np.ones(m.nv)) - L * L) < 1e-12 * L * L


def test_stiffness_leaves_only_the_boundary_flux_of_a_linear_function():
    """(K u)_i = int grad u . grad phi_i = boundary integral of (du/dn) phi_i for
    harmonic u: zero at interior vertices, -a h on the left edge, +a h on the
    right, -b h at the bottom, +b h at the top, half of each edge's value from
    both edges at a corner."""
    n, L = 8, L10
    m = fem.BoxMesh(n, L)
    h = L / n
    a, b = 0.9, -0.35
    Ku = fem.p1_stiffness(m) @ _linear(m, a, b, 2.0)
    i = np.arange(m.nv) % (n + 1)
    j = np.arange(m.nv) // (n + 1)
    ref = np.zeros(m.nv)
    for onb, val in ((i == 0, -a), (i == n, a), (j == 0, -b), (j == n, b)):
        corner = onb & (((i == 0) | (i == n)) & ((j == 0) | (j == n)))
        ref[onb & ~corner] += val * h
        ref[corner] += val * h / 2
    assert np.abs(Ku - ref).max() < 1e-13


def test_neumann_problem_converges_at_second_order():
    """(M + K) u_h = (f, phi_i) for -lap u + u = f with du/dn = 0 and
    u = cos(pi x/L) cos(pi y/L): the L^2 norm of the difference to the
    interpolant of u falls as h^2 (the maximum norm only as h^2 log(1/h))."""
    L = L10
    k = np.pi / L
    u = lambda x, y: np.cos(k * x) * np.cos(k * y)
    f = lambda x, y: (1.0 + 2.0 * k * k) * u(x, y)
    errs = []
    for n in (8, 16, 32, 64):
        m = fem.BoxMesh(n, L)
        M = fem.p1_mass(m)
        uh = solvers.sparse_solve(M + fem.p1_stiffness(m), fem.p1_load(m, f))
        xy = m.vertex_xy()
        e = uh - u(xy[:, 0], xy[:, 1])
        errs.append(np.sqrt(e @ (M @ e)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 1.95, (errs, rates)


def _box(n, L=L10):
    return S.Operators(n, box_length=L)


PB = dict(eps=0.1 ** 0.5, tau=1e-4, mobility=1.0, evap_rate=1.0)


@pytest.mark.parametrize("model", ["ch", "ch_ac"])
def test_step_conserves_the_phase_mass(model):
    n = 16
    ops, prm = _box(n), Params(**PB)
    f = inputs.box_state(n, L10, model, 1.0, 11)
    st = S.initial_state(ops, prm, model, f)
    out = S.step(ops, prm, model, st)
    m0, m1 = S.mass(ops, st["phi"][0]), S.mass(ops, out["phi"][0])
    assert abs(m1 - m0) <= 1e-12 * abs(m0)
    # the film's mass: half the box at about 1 (the interface row counts half)
    assert abs(m0 - 0.5 * L10 * L10) < 0.05 * L10 * L10


def test_constant_states_are_fixed_or_follow_the_reaction():
    """Constant phi and Phi: K annihilates constants, so phi stays, mu becomes
    f'(phi) and the vapour field takes one explicit reaction step
    Phi - tau gamma_v f_v'(phi, Phi)."""
    n = 8
    ops, prm = _box(n), Params(**PB)
    c, cv = 0.37, 0.6
    st = S.initial_state(ops, prm, "ch_ac", dict(phi=[np.full(ops.N, c)], Phi_v=np.full(ops.N, cv)))
    out = S.step(ops, prm, "ch_ac", st)
    assert np.abs(out["phi"][0] - c).max() < 1e-13
    assert np.abs(out["mu"][0] - pot.dfdphi_bin(c, cv)).max() < 1e-12
    ref = cv - prm.tau * prm.gamma_v * pot.dfdPhi_bin(c, cv)
    assert np.abs(out["Phi_v"] - ref).max() < 1e-13


def _perms(n):
    m = n + 1
    j, i = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    i, j = i.ravel(), j.ravel()
    transpose = j + m * i
    rotate = (n - i) + m * (n - j)
    return transpose, rotate


@pytest.mark.parametrize("which", [0, 1])
def test_step_commutes_with_the_mesh_symmetries(which):
    """The right-diagonal triangulation of the square is invariant under
    x <-> y and under the half turn about the centre; so is the step."""
    n = 12
    ops, prm = _box(n), Params(**PB)
    g = inputs.rng(5)
    phi = 0.5 + 0.1 * g.uniform(-1, 1, ops.N)
    Phi = 0.5 + 0.3 * g.uniform(-1, 1, ops.N)
    P = _perms(n)[which]
    a = S.step(ops, prm, "ch_ac", S.initial_state(ops, prm, "ch_ac", dict(phi=[phi], Phi_v=Phi)))
    b = S.step(ops, prm, "ch_ac", S.initial_state(ops, prm, "ch_ac", dict(phi=[phi[P]], Phi_v=Phi[P])))
    for x, y in ((a["phi"][0], b["phi"][0]), (a["mu"][0], b["mu"][0]), (a["Phi_v"], b["Phi_v"])):
        assert np.abs(x[P] - y).max() < 1e-11 * np.abs(x).max()


def test_small_steps_decrease_the_energy():
    """The discrete CH energy beta/2 phi^T K phi + sum (M 1)_i f(phi_i) falls
    along small steps from a noisy film (gradient flow with no-flux walls)."""
    n = 16
    ops, prm = _box(n), Params(**dict(PB, tau=1e-6))
    st = S.initial_state(ops, prm, "ch", inputs.box_state(n, L10, "ch", 0.5, 3))
    E = [S.energy_ch(ops, prm, st["phi"][0])]
    for _ in range(4):
        out = S.step(ops, prm, "ch", st)
        st = dict(st, phi=out["phi"], mu=out["mu"])
        E.append(S.energy_ch(ops, prm, st["phi"][0]))
    assert all(E[k + 1] < E[k] for k in range(4)), E


def test_direct_solvers_agree_and_the_fourier_solve_is_refused():
    n = 8
    ops, prm = _box(n), Params(**PB)
    st = S.initial_state(ops, prm, "ch_ac", inputs.box_state(n, L10, "ch_ac", 1.0, 4))
    a = S.step(ops, prm, "ch_ac", st, "dense")
    b = S.step(ops, prm, "ch_ac", st, "splu")
    assert np.abs(a["phi"][0] - b["phi"][0]).max() < 1e-12
    assert np.abs(a["Phi_v"] - b["Phi_v"]).max() < 1e-12
    with pytest.raises(ValueError):
        S.step(ops, prm, "ch_ac", st, "fft")


# ---------------------------------------------------------------- multigrid on the closed square


def test_box_prolongation_is_exact_on_linear_functions_and_nested():
    from oracle import multigrid as mg
    nf, L = 16, L10
    P = mg.prolongation_box(nf)
    fine, coarse = fem.BoxMesh(nf, L), fem.BoxMesh(nf // 2, L)
    lin = lambda xy: 0.4 * xy[:, 0] + 0.9 * xy[:, 1] - 2.0
    assert np.abs(P @ lin(coarse.vertex_xy()) - lin(fine.vertex_xy())).max() < 1e-12
    for form in (fem.p1_mass, fem.p1_stiffness):
        Af, Ac = form(fine), form(coarse)
        assert abs(P.T @ Af @ P - Ac).max() < 1e-13 * abs(Ac).max()


def test_box_vcycle_converges_and_is_symmetric():
    from oracle import multigrid as mg, precond as PC
    n = 32
    ops = _box(n)
    prm = Params(eps=0.1 ** 0.5, tau=1e-2, mobility=1.0)
    X = PC.matching_factor(ops.M, ops.K, prm)
    a, b = np.sqrt(prm.tau * prm.gamma / prm.beta), prm.tau * prm.gamma
    H = mg.Hierarchy(X, n, a=a, b=b, rho_cut=0.0, box_length=L10)
    assert H.sizes == [32, 16, 8, 4] and H.A[-1].shape == (25, 25)
    g = np.random.default_rng(2)
    x, y = g.standard_normal(ops.N), g.standard_normal(ops.N)
    assert abs(x @ mg.vcycle(H, y) - y @ mg.vcycle(H, x)) < 1e-10 * abs(x @ mg.vcycle(H, x))
    e = g.standard_normal(ops.N)
    e0 = np.linalg.norm(e)
    for _ in range(5):
        e = e - mg.vcycle(H, X @ e)
    assert (np.linalg.norm(e) / e0) ** (1 / 5) < 0.3


def test_level_cut_uses_the_mesh_width():
    """rho_l = 8 b / (a h_l^2): on a square of side L the rule cuts where the unit
    square cuts b / L^2."""
    from oracle import multigrid as mg
    sizes = mg.level_sizes(128)
    for a, b in ((0.03, 1e-4), (1.0, 1e-3), (2.0, 0.5)):
        assert mg.cut_level(sizes, a, b, length=L10) == mg.cut_level(sizes, a, b / L10 ** 2)
    assert mg.rho(2.0, 0.5, 64, 4.0) == 8 * 0.5 * 16 ** 2 / 2.0


# ---------------------------------------------------------------- evaporation flux at the top wall


def test_top_edge_load_integrates_and_carries_inhomogeneous_neumann_data():
    """b_i = int_top g phi_i ds: sums to int_top g and integrates linear g
    exactly; with it, (M + K) u_h = (f, phi_i) + j b solves -lap u + u = f with
    du/dn = j on the top wall and 0 elsewhere: u = y^2 (f = y^2 - 2, j = 2 L)
    is reached at second order."""
    L = L10
    m = fem.BoxMesh(12, L)
    b = fem.top_edge_load(m)
    assert abs(b.sum() - L) < 1e-13 and np.count_nonzero(b) == 13
    xy = m.vertex_xy()
    bx = fem.top_edge_load(m, lambda x: 1.0 + 0.3 * x)
    assert abs(bx @ xy[:, 0] - (L * L / 2 + 0.3 * L ** 3 / 3)) < 1e-11
    errs = []
    for n in (8, 16, 32, 64):
        m = fem.BoxMesh(n, L)
        M = fem.p1_mass(m)
        rhs = fem.p1_load(m, lambda x, y: y * y - 2.0) + 2.0 * L * fem.top_edge_load(m)
        uh = solvers.sparse_solve(M + fem.p1_stiffness(m), rhs)
        e = uh - m.vertex_xy()[:, 1] ** 2
        errs.append(np.sqrt(e @ (M @ e)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 1.95, (errs, rates)


def test_top_flux_enters_linearly_conserves_mass_and_draws_phase_to_the_wall():
    """The flux j_out = k (phi^k(x_ref) - phi_inf) only loads the mu equation:
    no flux when phi(x_ref) = phi_inf, a response linear in k, the phase mass
    unchanged (d mu / dn = 0 on every wall), and for j_out > 0 a lower mu at
    the wall that draws phase towards it (d phi / dn > 0 there)."""
    n = 16
    ops = _box(n)
    base = Params(**PB)
    st = S.initial_state(ops, base, "ch_ac", inputs.box_state(n, L10, "ch_ac", 0.5, 6))
    ref = n // 2 + (n + 1) * n
    phi_ref = st["phi"][0][ref]
    plain = S.step(ops, base, "ch_ac", st)
    same = S.step(ops, Params(**dict(PB, top_flux=3.0, flux_inf=phi_ref)), "ch_ac", st)
    assert np.array_equal(same["phi"][0], plain["phi"][0])
    d = []
    for k in (1.0, 2.0):
        out, sysr = S.step(ops, Params(**dict(PB, top_flux=k, flux_inf=phi_ref - 0.2)), "ch_ac", st,
                           return_systems=True)
        assert abs(sysr["j_out"] - 0.2 * k) < 1e-15
        d.append(out["phi"][0] - plain["phi"][0])
        assert abs(S.mass(ops, out["phi"][0]) - S.mass(ops, plain["phi"][0])) < 1e-12 * L10 * L10
        assert np.array_equal(out["Phi_v"], plain["Phi_v"])  # the vapour equation is untouched
    # linear up to the rounding of the two O(1) solutions whose difference d is
    assert np.abs(d[1] - 2.0 * d[0]).max() < 1e-12 * np.abs(plain["phi"][0]).max()
    assert np.abs(d[1]).max() > 1e-5
    top = np.arange(ops.N) >= (n + 1) * n
    assert d[0][top].sum() > 0 and d[0][~top].sum() < 0
    with pytest.raises(ValueError):
        S.step(S.Operators(n), Params(**dict(PB, top_flux=1.0)), "ch", {"phi": [np.zeros(n * n)],
                                                                      "mu": [np.zeros(n * n)]})
