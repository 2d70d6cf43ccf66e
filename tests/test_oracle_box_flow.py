"""Pins of the oracle's flow models on the closed square [0, L]^2: the
Taylor-Hood spaces with the no-slip walls of eq. (bc) (velocity zero on every
wall) and the natural conditions of the phase fields.

Pinned against the mesh's own geometry (P2 ids at the edge midpoints, the
unused ids of the padded numbering), exact forms on linear fields, a
manufactured solution of the Oseen system with no-slip walls (velocity at
third order, pressure at second, forcing derived symbolically), and step
invariants (walls held at zero, discrete incompressibility, the mass balance
of the convected phases, dense = sparse solves)."""
import numpy as np
import pytest
import scipy.sparse as sp
import sympy as sy

from oracle import fem, solvers, step as S, systems
from oracle.systems import Params
from paper_2501_11767_amd import inputs

L2 = 2.0


@pytest.mark.parametrize("n", [4, 10])
def test_p2_ids_sit_at_the_edge_midpoints(n):
    m = fem.BoxMesh(n, L2)
    xy2 = m.p2_xy()
    assert np.array_equal(xy2, inputs.box_p2_coords(n, L2))
    for k, (a, b) in zip((3, 4, 5), ((1, 2), (0, 2), (0, 1))):
        assert np.allclose(xy2[m.tri2[:, k]], 0.5 * (m.xy[:, a] + m.xy[:, b]))
    assert np.allclose(xy2[m.tri2[:, :3]], m.xy)
    used = np.zeros(4 * m.nv, bool)
    used[m.tri2.ravel()] = True
    assert used.sum() == (2 * n + 1) ** 2 and np.array_equal(~used, inputs.box_p2_unused(n))
    fixed = m.p2_fixed()
    assert fixed.sum() == 12 * n + 3  # 8n wall nodes and 4n + 3 unused ids
    assert np.array_equal(fixed, inputs.box_p2_wall(n) | inputs.box_p2_unused(n))
    w = xy2[fixed & used]
    on_wall = (np.isclose(w[:, 0], 0) | np.isclose(w[:, 0], L2) | np.isclose(w[:, 1], 0) | np.isclose(w[:, 1], L2))
    assert on_wall.all()
    inner = xy2[~fixed]
    assert np.all((inner > 1e-12) & (inner < L2 - 1e-12))


def test_p2_forms_on_linear_fields():
    n = 6
    m = fem.BoxMesh(n, L2)
    xy2 = m.p2_xy()
    one = np.ones(4 * m.nv)
    assert abs(one @ (fem.p2_mass(m) @ one) - L2 * L2) < 1e-13
    # B = -int q div u: the P2 interpolant of u = (x, 0) has div u = 1
    B = fem.divergence_matrix(m)
    u = np.concatenate([xy2[:, 0], np.zeros(4 * m.nv)])
    assert np.abs(B @ u + fem.p1_mass(m) @ np.ones(m.nv)).max() < 1e-13
    # K_sym annihilates rigid translations
    Ks = fem.p2_sym_stiffness(m, 1.3)
    assert np.abs(Ks @ np.concatenate([one, 0 * one])).max() < 1e-12


def _mms():
    x, y, Ls = sy.symbols("x y L", positive=True)
    psi = sy.sin(sy.pi * x / Ls) ** 2 * sy.sin(sy.pi * y / Ls) ** 2
    u, v = sy.diff(psi, y), -sy.diff(psi, x)
    p = sy.cos(sy.pi * x / Ls) * sy.cos(sy.pi * y / Ls)
    return x, y, Ls, u, v, p


def test_mms_oseen_no_slip_orders():
    """(rho/tau) M v + J(w) v + K_sym v + B^T p = (f, zeta), B v = 0, v = 0 on
    the walls, for v = curl psi, psi = sin^2(pi x/L) sin^2(pi y/L) (v vanishes on
    the walls), p = cos(pi x/L) cos(pi y/L) (mean zero), constant w: velocity
    in L^2 at order 3, pressure at order 2."""
    x, y, Ls, u, v, p = _mms()
    prm = Params(eps=0.1, tau=0.05, viscosity=0.7, rho=1.0)
    wa, wb = 0.5, -0.25
    k, eta = prm.rho / prm.tau, prm.viscosity
    lap = lambda f: sy.diff(f, x, 2) + sy.diff(f, y, 2)
    fx = k * u + wa * sy.diff(u, x) + wb * sy.diff(u, y) - eta * lap(u) + sy.diff(p, x)
    fy = k * v + wa * sy.diff(v, x) + wb * sy.diff(v, y) - eta * lap(v) + sy.diff(p, y)
    num = lambda e: sy.lambdify((x, y), e.subs(Ls, L2), "numpy")
    U, V, Pf, FX, FY = (num(e) for e in (u, v, p, fx, fy))
    ev, ep = [], []
    for n in (8, 16, 32):
        ops = S.Operators(n, need_p2=True, box_length=L2)
        m = ops.mesh
        w = np.zeros((2, 4 * m.nv))
        w[0], w[1] = wa, wb
        J = fem.p2_convection(m, w)
        Avel = systems.oseen_velocity_block(ops.Mv, J, ops.Ksym(eta), prm)
        rhs = fem.p2_load_vec(m, FX, FY)
        vel, pr, _ = solvers.bordered_oseen_solve(Avel, ops.B, ops.M, rhs, fixed=ops.vfixed)
        assert np.all(vel[ops.vfixed] == 0.0)
        xy2 = m.p2_xy()
        used = ~inputs.box_p2_unused(n)
        ex = np.where(used, U(xy2[:, 0], xy2[:, 1]), 0.0)
        ey = np.where(used, V(xy2[:, 0], xy2[:, 1]), 0.0)
        eu = vel - np.concatenate([ex, ey])
        Mv2 = sp.block_diag([ops.Mv, ops.Mv])
        ev.append(np.sqrt(eu @ (Mv2 @ eu)))
        xy = m.vertex_xy()
        epp = pr - Pf(xy[:, 0], xy[:, 1])
        epp -= (np.ones(m.nv) @ (ops.M @ epp)) / L2 ** 2
        ep.append(np.sqrt(epp @ (ops.M @ epp)))
    rv = np.log2(np.array(ev[:-1]) / np.array(ev[1:]))
    rp = np.log2(np.array(ep[:-1]) / np.array(ep[1:]))
    assert rv.min() > 2.7 and rp.min() > 1.8, (ev, ep, rv, rp)


PF = dict(eps=0.3, tau=1e-3, mobility=1.0, evap_rate=0.5, viscosity=0.5, alpha=1e-3)


@pytest.mark.parametrize("model", ["ternary", "quaternary"])
def test_flow_step_keeps_the_walls_and_incompressibility(model):
    n = 8
    kw = dict(betas=(2e-3, 2e-3, 1e-2, 4e-2)) if model == "quaternary" else {}
    prm = Params(**PF, **kw)
    ops = S.Operators(n, need_p2=True, box_length=L2)
    st = S.initial_state(ops, prm, model, inputs.box_state(n, L2, model, 0.33, 3))
    assert np.abs(np.asarray(st["vel"])[:, ops.mesh.p2_fixed()]).max() == 0.0
    a = S.step(ops, prm, model, st, "dense")
    b = S.step(ops, prm, model, st, "splu")
    assert np.abs(a["vel"] - b["vel"]).max() < 1e-12 * np.abs(a["vel"]).max()
    assert np.abs(a["p"] - b["p"]).max() < 1e-9 * np.abs(a["p"]).max()
    vel = b["vel"].ravel()
    assert np.all(vel[ops.vfixed] == 0.0) and np.abs(vel).max() > 0
    assert np.abs(ops.B @ vel).max() < 1e-12 * np.abs(vel).max()
    assert abs(np.ones(ops.N) @ (ops.M @ b["p"])) < 1e-12 * np.abs(b["p"]).max()
    # convected phases: 1^T M (phi^1 - phi^0) + tau 1^T C phi^1 = 0 (K 1 = 0)
    C = fem.p1_convection(ops.mesh, st["vel"])
    one = np.ones(ops.N)
    for i in range(len(st["phi"])):
        r = one @ (ops.M @ (b["phi"][i] - st["phi"][i])) + prm.tau * one @ (C @ b["phi"][i])
        assert abs(r) < 1e-12 * abs(one @ (ops.M @ st["phi"][i])), i


def test_stream_velocity_is_discretely_near_solenoidal_and_zero_on_the_walls():
    n = 16
    m = fem.BoxMesh(n, L2)
    vel = inputs.box_stream_velocity(n, L2, 4, amp=0.05)
    assert np.abs(vel[:, m.p2_fixed()]).max() == 0.0
    B = fem.divergence_matrix(m)
    d = B @ vel.ravel()
    # interpolation error only: O(h^2) relative to the gradient scale
    assert np.abs(d).max() < 0.05 * (L2 / n) ** 2 * 10


def test_p1_to_p2_interpolation_on_any_numbering():
    """The mesh-generic P1 -> P2 interpolation: the periodic formula on the
    periodic square, exact for linear fields at the closed square's P2 nodes,
    zero at its unused ids."""
    n = 6
    g = np.random.default_rng(0)
    m = fem.Mesh(n)
    u = g.standard_normal(m.nv)
    assert np.abs(fem.p2_eval_p1_interp_mesh(m, u) - fem.p2_eval_p1_interp(n, u)).max() == 0.0
    b = fem.BoxMesh(n, L2)
    xy, xy2 = b.vertex_xy(), b.p2_xy()
    a = np.array([0.7, -1.3])
    got = fem.p2_eval_p1_interp_mesh(b, xy @ a + 0.2)
    unused = inputs.box_p2_unused(n)
    assert np.abs(got[~unused] - (xy2[~unused] @ a + 0.2)).max() < 1e-14 and np.all(got[unused] == 0.0)


def test_variable_density_step_on_the_closed_square():
    """Variable density with Picard passes on the closed square: walls held,
    discrete incompressibility, the convected phases' mass balance, dense =
    sparse; the density changes the step (against rho = 1)."""
    n = 8
    prm = Params(**PF, rho_pure=(1.3, 0.8, 1.0), picard=3)
    ops = S.Operators(n, need_p2=True, box_length=L2)
    st = S.initial_state(ops, prm, "ternary", inputs.box_state(n, L2, "ternary", 0.33, 3))
    a = S.step(ops, prm, "ternary", st, "dense")
    b = S.step(ops, prm, "ternary", st, "splu")
    assert np.abs(a["vel"] - b["vel"]).max() < 1e-11 * np.abs(a["vel"]).max()
    vel = b["vel"].ravel()
    assert np.all(vel[ops.vfixed] == 0.0) and np.abs(ops.B @ vel).max() < 1e-12 * np.abs(vel).max()
    C = fem.p1_convection(ops.mesh, st["vel"])
    one = np.ones(ops.N)
    for i in range(2):
        r = one @ (ops.M @ (b["phi"][i] - st["phi"][i])) + prm.tau * one @ (C @ b["phi"][i])
        assert abs(r) < 1e-12 * abs(one @ (ops.M @ st["phi"][i])), i
    c = S.step(ops, Params(**PF, picard=3), "ternary", st, "splu")
    assert np.abs(c["vel"] - b["vel"]).max() > 1e-6 * np.abs(b["vel"]).max()
