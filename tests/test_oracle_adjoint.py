"""Pins of the oracle's discrete adjoint (differentiation form).

Each building block is checked against something other than itself: Hessian
entries against central differences of the first derivatives (and the mixed
partials against a different function's derivative), each vector-Jacobian
product against the forward assembly by a dot-product test (exact for forms
linear or quadratic in the differentiated argument), one reverse step against
central differences of the step map, and the whole gradient against central
differences of the loss with direct solves.
"""
import numpy as np
import pytest

from oracle import adjoint as AD, fem, potential as pot, step as S
from oracle.systems import Params
from paper_2501_11767_amd import inputs


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("potential", ["quartic", "flory_huggins"])
def test_hessian_matches_central_differences(seed, potential):
    """Second derivatives against central differences of the first
    derivatives, and the first derivatives against central differences of the
    density itself (so a wrong term anywhere in the chain fails).  The fitted
    quartic is also checked against its separately written reduced form."""
    g = np.random.default_rng(seed)
    pp, pn, Phi = g.uniform(0.05, 0.6, 50), g.uniform(0.05, 0.35, 50), g.uniform(-0.1, 1.1, 50)
    prm = Params(eps=0.02, tau=1e-3, potential=None if potential == "quartic" else pot.FloryHuggins())
    H = AD.hess_ter(pp, pn, Phi, prm)
    T = lambda a, b, c: S.ternary_potential(prm, a, b, c)
    h = 1e-6
    d = lambda f: (f(h) - f(-h)) / (2 * h)
    first = {
        "dp": d(lambda t: T(pp + t, pn, Phi)["f"]),
        "dn": d(lambda t: T(pp, pn + t, Phi)["f"]),
        "fv": d(lambda t: T(pp, pn, Phi + t)["f"]),
    }
    t0 = T(pp, pn, Phi)
    for k, fd in first.items():
        assert np.abs(t0[k] - fd).max() <= 1e-7 * (1 + np.abs(fd).max()), k
    checks = {
        "pp": d(lambda t: T(pp + t, pn, Phi)["dp"]),
        "pn": d(lambda t: T(pp, pn + t, Phi)["dp"]),
        "nn": d(lambda t: T(pp, pn + t, Phi)["dn"]),
        "pP": d(lambda t: T(pp, pn, Phi + t)["dp"]),
        "nP": d(lambda t: T(pp, pn, Phi + t)["dn"]),
        "vp": d(lambda t: T(pp + t, pn, Phi)["fv"]),
        "vn": d(lambda t: T(pp, pn + t, Phi)["fv"]),
        "vP": d(lambda t: T(pp, pn, Phi + t)["fv"]),
        "sp": d(lambda t: T(pp + t, pn, Phi)["fs"]),
        "sn": d(lambda t: T(pp, pn + t, Phi)["fs"]),
        "sP": d(lambda t: T(pp, pn, Phi + t)["fs"]),
    }
    for k, fd in checks.items():
        assert np.abs(H[k] - fd).max() <= 1e-7 * (1 + np.abs(fd).max()), k
    # mixed partials of f from two different first-derivative functions
    other = d(lambda t: T(pp + t, pn, Phi)["dn"])
    assert np.abs(H["pn"] - other).max() <= 1e-7 * (1 + np.abs(other).max())
    assert np.abs(H["vp"] - checks["pP"]).max() <= 1e-7 * (1 + np.abs(H["vp"]).max())
    if potential == "quartic":
        dp, dn = pot.dfdphi_ter(pp, pn, Phi)
        for a, b in ((t0["f"], pot.f_ter(pp, pn, Phi)), (t0["dp"], dp), (t0["dn"], dn),
                     (t0["fv"], pot.dfdPhi_ter(pp, pn, Phi)), (t0["fs"], pot.dfdphis_ter(1 - pp - pn, Phi))):
            assert np.abs(a - b).max() <= 1e-14 * (1 + np.abs(b).max())


@pytest.fixture(scope="module")
def mesh8():
    return fem.Mesh(8)


def test_p1_convection_vjp_dot_product(mesh8):
    m = mesh8
    g = np.random.default_rng(3)
    eta, x = g.standard_normal(m.nv), g.standard_normal(m.nv)
    dv = g.standard_normal((2, 4 * m.nv))
    lhs = eta @ (fem.p1_convection(m, dv) @ x)
    rhs = np.sum(AD.p1_conv_vjp(m, eta, x) * dv)
    assert _rel(rhs, lhs) < 1e-12


def test_p2_convection_vjp_dot_product(mesh8):
    m = mesh8
    g = np.random.default_rng(4)
    xi, u = g.standard_normal((2, 4 * m.nv)), g.standard_normal((2, 4 * m.nv))
    dw, dc = g.standard_normal((2, 4 * m.nv)), g.standard_normal((m.ne, 2))
    J = fem.p2_convection(m, dw, dc)
    lhs = sum(xi[c] @ (J @ u[c]) for c in range(2))
    gw, gc = AD.p2_conv_vjp(m, xi, u)
    rhs = np.sum(gw * dw) + np.sum(gc * dc)
    assert _rel(rhs, lhs) < 1e-12


def test_grad_transpose_dot_product(mesh8):
    m = mesh8
    g = np.random.default_rng(5)
    u, ge = g.standard_normal(m.nv), g.standard_normal((m.ne, 2))
    assert _rel(np.sum(AD.grad_T(m, ge) * u), np.sum(ge * fem.p1_grad(m, u))) < 1e-12


def test_korteweg_vjp_exact_for_quadratic_load(mesh8):
    m = mesh8
    g = np.random.default_rng(6)
    us = [g.standard_normal(m.nv) for _ in range(3)]
    betas = [0.3, 0.7, 1.9]
    xi = g.standard_normal(8 * m.nv)
    F = lambda fs: fem.korteweg_load(m, [fem.p1_grad(m, u) for u in fs], betas)
    vj = AD.korteweg_vjp(m, xi, us, betas)
    for i in range(3):
        du = g.standard_normal(m.nv)
        plus = [u + (du if j == i else 0) for j, u in enumerate(us)]
        minus = [u - (du if j == i else 0) for j, u in enumerate(us)]
        # F quadratic in u_i: the central difference with unit step is exact
        lhs = xi @ (F(plus) - F(minus)) / 2.0
        assert _rel(vj[i] @ du, lhs) < 1e-11


def _state(n, prm, seed=21):
    f = inputs.initial_state(n, "ternary", 0.3, seed)
    ops = S.Operators(n, need_p2=True)
    return ops, S.initial_state(ops, prm, "ternary", f)


def _flat(st):
    return np.concatenate([st["phi"][0], st["phi"][1], st["mu"][0], st["mu"][1], st["mu_s"],
                           st["Phi_v"], st["vel"].ravel(), st["p"]])


def _unflat(x, n, N=None):
    N = n * n if N is None else N
    o = 0

    def take(k):
        nonlocal o
        o += k
        return x[o - k:o]
    return dict(phi=[take(N), take(N)], mu=[take(N), take(N)], mu_s=take(N), Phi_v=take(N),
                vel=take(8 * N).reshape(2, 4 * N), p=take(N))


@pytest.mark.parametrize("potential", [None, "flory_huggins"])
def test_step_vjp_matches_central_differences(potential):
    """<lambda^{k+1}, (ds^{k+1}/ds^k) ds> and <lambda^{k+1}, ds^{k+1}/dtheta> by
    central differences of the direct-solve step, against the reverse step;
    alpha = 0.1 so that the chemical-potential path into the Oseen operator is
    visible.  Both densities: the fitted quartic and Flory-Huggins."""
    n = 8
    base = dict(eps=0.05, tau=2e-5, mobility=1.3, evap_rate=0.4, viscosity=1.0, alpha=0.1)
    if potential:
        base["potential"] = pot.FloryHuggins()
    prm = Params(**base)
    ops, st = _state(n, prm)
    g = np.random.default_rng(8)
    lam1 = AD.zero_adjoint(n * n)
    for i in range(2):
        lam1["phi"][i] = g.standard_normal(n * n)
        lam1["mu"][i] = g.standard_normal(n * n)
    lam1["mu_s"] = g.standard_normal(n * n)
    lam1["Phi_v"] = g.standard_normal(n * n)
    lam1["vel"] = g.standard_normal((2, 4 * n * n))
    lam0, dth = AD.step_vjp(ops, prm, st, AD.next_state(S.step(ops, prm, "ternary", st)), lam1)
    L1 = _flat(lam1)
    fwd = lambda p, s: _flat(AD.next_state(S.step(ops, p, "ternary", s)))
    x0 = _flat(st)
    for seed in (1, 2):
        dx = np.random.default_rng(seed).standard_normal(x0.size)
        dx[-n * n:] = 0.0  # the pressure of step k enters nothing
        h = 1e-5
        fd = L1 @ (fwd(prm, _unflat(x0 + h * dx, n)) - fwd(prm, _unflat(x0 - h * dx, n))) / (2 * h)
        assert _rel(_flat(lam0) @ dx, fd) < 1e-6, seed
    # relative steps of 1e-3: smaller ones are dominated by rounding in the
    # difference of two O(1) inner products
    for j, key in enumerate(("eps", "mobility", "evap_rate")):
        h = 1e-3 * base[key]
        pp = Params(**dict(base, **{key: base[key] + h}))
        pm = Params(**dict(base, **{key: base[key] - h}))
        fd = L1 @ (fwd(pp, st) - fwd(pm, st)) / (2 * h)
        assert _rel(dth[j], fd) < 1e-6, key


def test_gradient_matches_central_differences_of_the_loss():
    """Fourth-order central differences (relative step 1e-3, truncation error
    O(h^4)) of the loss computed with direct solves."""
    n, steps = 8, 4
    ref = dict(eps=0.05, tau=5e-5, mobility=2.0, evap_rate=0.2, viscosity=1.0, alpha=1e-8)
    th0 = dict(ref, eps=0.045, mobility=1.5, evap_rate=0.15)
    ops, st0 = _state(n, Params(**ref), seed=33)
    target = AD.rollout(ops, Params(**ref), st0, steps)[-1]["phi"]
    L, grad = AD.gradient(ops, Params(**th0), st0, target, steps)
    assert L > 0

    def Lat(key, v):
        return AD.loss(ops, AD.rollout(ops, Params(**dict(th0, **{key: v})), st0, steps)[-1], target)

    for j, key in enumerate(("eps", "mobility", "evap_rate")):
        x, h = th0[key], 1e-3 * th0[key]
        fd = (-Lat(key, x + 2 * h) + 8 * Lat(key, x + h) - 8 * Lat(key, x - h) + Lat(key, x - 2 * h)) / (12 * h)
        assert _rel(grad[j], fd) < 1e-6, (key, grad[j], fd)
    # at the reference parameters the loss and its gradient vanish
    L0, g0 = AD.gradient(ops, Params(**ref), st0, target, steps)
    assert L0 == 0.0 and np.all(g0 == 0.0)


def test_step_vjp_on_the_closed_square_matches_central_differences():
    """The reverse step on the closed square (no-slip unknowns left out of the
    adjoint Oseen solve) against central differences of the direct-solve step,
    state and parameters; the perturbation touches every input, walls
    included."""
    n, Lb = 6, 2.0
    base = dict(eps=0.1, tau=1e-4, mobility=1.3, evap_rate=0.4, viscosity=1.0, alpha=0.1)
    prm = Params(**base)
    ops = S.Operators(n, need_p2=True, box_length=Lb)
    st = S.initial_state(ops, prm, "ternary", inputs.box_state(n, Lb, "ternary", 0.33, 5))
    N = ops.N
    g = np.random.default_rng(8)
    lam1 = AD.zero_adjoint(N)
    for i in range(2):
        lam1["phi"][i] = g.standard_normal(N)
        lam1["mu"][i] = g.standard_normal(N)
    lam1["mu_s"] = g.standard_normal(N)
    lam1["Phi_v"] = g.standard_normal(N)
    lam1["vel"] = g.standard_normal((2, 4 * N))
    lam0, dth = AD.step_vjp(ops, prm, st, AD.next_state(S.step(ops, prm, "ternary", st)), lam1)
    L1 = _flat(lam1)
    fwd = lambda p, s: _flat(AD.next_state(S.step(ops, p, "ternary", s)))
    x0 = _flat(st)
    for seed in (1, 2):
        dx = np.random.default_rng(seed).standard_normal(x0.size)
        dx[-N:] = 0.0  # the pressure of step k enters nothing
        h = 1e-5
        fd = L1 @ (fwd(prm, _unflat(x0 + h * dx, n, N)) - fwd(prm, _unflat(x0 - h * dx, n, N))) / (2 * h)
        assert _rel(_flat(lam0) @ dx, fd) < 1e-6, seed
    for j, key in enumerate(("eps", "mobility", "evap_rate")):
        h = 1e-3 * base[key]
        pp = Params(**dict(base, **{key: base[key] + h}))
        pm = Params(**dict(base, **{key: base[key] - h}))
        fd = L1 @ (fwd(pp, st) - fwd(pm, st)) / (2 * h)
        assert _rel(dth[j], fd) < 1e-6, key
