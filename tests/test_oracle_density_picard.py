"""Pins of the oracle's variable-density Oseen step (rho^k = sum_i rho_i
phi_i^k in the mass and convection terms of eq. (matrixns)) and of the Picard
passes of the Oseen solve (the outer iteration the Newton remark after eq.
(linearnav) alludes to), against closed forms, analytic integrals, the
constant-density step and the nonlinear fixed point they converge to."""
import numpy as np
import pytest

from oracle import fem, step as S, systems
from oracle.systems import Params
from paper_2501_11767_amd import inputs

BASE = dict(eps=0.04, tau=1e-4, mobility=1.0, evap_rate=0.1, viscosity=1.0, alpha=1e-8, rho=1.0)


def _g(x, y):
    return np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.3


def _r(x, y):
    return 1.0 + 0.5 * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y)


def _vertex_values(n, f):
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return f(i.ravel() / n, j.ravel() / n)


def _p2_values(n, f):
    """f at the P2 nodes: vertices, then horizontal, vertical, diagonal edge midpoints."""
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x, y = i.ravel() / n, j.ravel() / n
    h = 1.0 / n
    return np.concatenate([f(x, y), f(x + h / 2, y), f(x, y + h / 2), f(x + h / 2, y + h / 2)])


def _ref_integral(f, m=64):
    """int_[0,1]^2 f by a tensor Gauss-Legendre rule on an m x m grid of cells."""
    t, w = np.polynomial.legendre.leggauss(8)
    t, w = 0.5 * (t + 1), 0.5 * w
    c = np.arange(m) / m
    xs = (c[:, None] + t[None, :] / m).ravel()
    ws = np.tile(w / m, m)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    return float(np.einsum("i,j,ij->", ws, ws, f(X, Y)))


@pytest.mark.parametrize("n", [8, 16])
def test_weighted_masses_reduce_to_the_masses_and_integrate_rho(n):
    m = fem.Mesh(n)
    rho = _vertex_values(n, _r)
    M2, M1 = fem.p2_mass_weighted(m, rho), fem.p1_mass_weighted(m, rho)
    # rho = 1: the unweighted masses
    one = np.ones(n * n)
    assert abs(fem.p2_mass_weighted(m, one) - fem.p2_mass(m)).max() < 1e-15
    assert abs(fem.p1_mass_weighted(m, one) - fem.p1_mass(m)).max() < 1e-15
    # 1^T M_rho 1 = int I_1 rho = h^2 sum_i rho_i (every vertex hat integrates to h^2)
    h2 = 1.0 / (n * n)
    assert abs(np.ones(4 * n * n) @ (M2 @ np.ones(4 * n * n)) - h2 * rho.sum()) < 1e-14
    assert abs(one @ (M1 @ one) - h2 * rho.sum()) < 1e-14
    # symmetric, linear in rho, positive definite for positive rho
    assert abs(M2 - M2.T).max() < 1e-18 and abs(M1 - M1.T).max() < 1e-18
    r2 = _vertex_values(n, lambda x, y: np.cos(2 * np.pi * (x + y)))
    lin = fem.p2_mass_weighted(m, 2.0 * rho - 3.0 * r2) - (2.0 * M2 - 3.0 * fem.p2_mass_weighted(m, r2))
    assert abs(lin).max() < 1e-16
    assert np.linalg.eigvalsh(M1.toarray()).min() > 0


def test_weighted_mass_converges_to_the_weighted_integral():
    """u^T M_rho u -> int r g^2 for the P2 interpolant u of g and the P1
    interpolant of r (second order at least: the interpolation errors)."""
    ref = _ref_integral(lambda x, y: _r(x, y) * _g(x, y) ** 2)
    errs = []
    for n in (8, 16, 32):
        m = fem.Mesh(n)
        u = _p2_values(n, _g)
        errs.append(abs(u @ (fem.p2_mass_weighted(m, _vertex_values(n, _r)) @ u) - ref))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.9, (errs, rates)
    assert errs[-1] < 1e-3 * abs(ref)


def _state(n, prm, seed=2):
    ops = S.Operators(n, need_p2=True)
    f = inputs.initial_state(n, "ternary", 0.3, seed)
    return ops, S.initial_state(ops, prm, "ternary", f)


def test_equal_pure_densities_reproduce_the_constant_density_step():
    n = 16
    ops, st = _state(n, Params(**BASE))
    ref = S.step(ops, Params(**dict(BASE, rho=1.7)), "ternary", st)
    got = S.step(ops, Params(**dict(BASE, rho=9.0, rho_pure=(1.7, 1.7, 1.7))), "ternary", st)
    # the same system up to the rounding of rho^k = sum_i 1.7 phi_i; the mean-zero
    # pressure of the saddle point amplifies rounding about 1e3-fold at n = 16
    assert np.abs(got["vel"] - ref["vel"]).max() <= 1e-12 * np.abs(ref["vel"]).max()
    assert np.abs(got["p"] - ref["p"]).max() <= 1e-9 * np.abs(ref["p"]).max()


def test_density_field_enters_mass_and_convection():
    n = 16
    prm = Params(**dict(BASE, rho_pure=(1.2, 0.8, 1.0)))
    ops, st = _state(n, prm)
    st["vel"] = inputs.stream_velocity(n, 3, amp=0.02)
    out, sysr = S.step(ops, prm, "ternary", st, return_systems=True)
    rho = systems.density(prm, st["phi"][0], st["phi"][1])
    assert np.allclose(rho, 1.2 * st["phi"][0] + 0.8 * st["phi"][1] + (1 - st["phi"][0] - st["phi"][1]))
    # the velocity block's mass is the weighted one
    Mr = fem.p2_mass_weighted(ops.mesh, rho)
    assert abs(sysr["ns_Mrho"] - Mr).max() < 1e-18
    # the solution solves the recorded system and differs from the constant-density one
    const = S.step(ops, Params(**BASE), "ternary", st)
    assert np.linalg.norm(out["vel"] - const["vel"]) > 1e-6 * np.linalg.norm(const["vel"])
    A = systems.oseen_matrix(sysr["ns_A"], ops.B)
    x = np.concatenate([out["vel"].ravel(), out["p"]])
    b = np.concatenate([sysr["ns_rhs"], np.zeros(n * n)])
    assert np.linalg.norm(A @ x - b) <= 1e-11 * np.linalg.norm(b)


@pytest.mark.parametrize("rho_pure", [None, (1.2, 0.8, 1.0)])
def test_picard_passes_converge_to_the_nonlinear_fixed_point(rho_pure):
    """Picard passes: one pass is the linear scheme; with a strong flow the
    changes between passes contract, and the converged velocity solves the
    Oseen system convected by itself (the implicit convection)."""
    n = 16
    base = dict(BASE, tau=2e-3, viscosity=0.05, rho_pure=rho_pure)
    ops, st = _state(n, Params(**base))
    st["vel"] = inputs.stream_velocity(n, 3, amp=0.05)
    lin = S.step(ops, Params(**base), "ternary", st)
    one = S.step(ops, Params(**dict(base, picard=1)), "ternary", st)
    assert np.array_equal(lin["vel"], one["vel"])
    vs = [st["vel"]]
    for k in range(1, 7):
        vs.append(S.step(ops, Params(**dict(base, picard=k)), "ternary", st)["vel"])
    d = [np.linalg.norm(vs[i + 1] - vs[i]) for i in range(len(vs) - 1)]
    assert all(d[i + 1] < 0.5 * d[i] for i in range(1, len(d) - 1)), d
    out, sysr = S.step(ops, Params(**dict(base, picard=50, picard_tol=1e-13)), "ternary", st,
                       return_systems=True)
    assert sysr["ns_passes"] < 50
    # fixed point: J formed with the solution itself
    prm = Params(**base)
    rho_k = systems.density(prm, st["phi"][0], st["phi"][1])
    J = fem.p2_convection(ops.mesh, S.convecting_field(n, prm, rho_k, out["vel"]), sysr["ns_w_const"])
    Mr = None if rho_k is None else fem.p2_mass_weighted(ops.mesh, rho_k)
    A = systems.oseen_matrix(systems.oseen_velocity_block(ops.Mv, J, ops.Ksym(prm.viscosity), prm, Mr), ops.B)
    x = np.concatenate([out["vel"].ravel(), out["p"]])
    b = np.concatenate([sysr["ns_rhs"], np.zeros(n * n)])
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)
    # and it is not the linear scheme's answer
    assert np.linalg.norm(out["vel"] - lin["vel"]) > 1e-8 * np.linalg.norm(lin["vel"])


def test_picard_tolerance_stops_early_and_the_reverse_step_refuses():
    from oracle import adjoint as AD
    n = 8
    base = dict(BASE, tau=2e-3, viscosity=0.05)
    ops, st = _state(n, Params(**base))
    st["vel"] = inputs.stream_velocity(n, 3, amp=0.05)
    _, s1 = S.step(ops, Params(**dict(base, picard=40, picard_tol=1e-6)), "ternary", st, return_systems=True)
    _, s2 = S.step(ops, Params(**dict(base, picard=40, picard_tol=1e-12)), "ternary", st, return_systems=True)
    assert 2 <= s1["ns_passes"] < s2["ns_passes"] < 40
    st1 = AD.next_state(S.step(ops, Params(**base), "ternary", st))
    for bad in (dict(picard=2), dict(rho_pure=(1.0, 1.0, 1.0))):
        with pytest.raises(NotImplementedError):
            AD.step_vjp(ops, Params(**dict(base, **bad)), st, st1, AD.zero_adjoint(n * n))
