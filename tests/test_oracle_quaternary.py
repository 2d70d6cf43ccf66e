"""Pins of the oracle's quaternary model: polymer, NFA and solvent phases with
the air eliminated (phi_a = 1 - phi_p - phi_N - phi_s, section "Numerical
results"), the fitted quartic of eq. (appPotential) with its air terms, a
gradient coefficient per phase, mu_a from eq. (airdisc).

Pinned against central differences of the density, the ternary reduction at
zero air (the same quartic, other variables), exact conservation of every
phase's mass, constant states, the polymer/NFA symmetry of the density, and
the energy decay of a small step."""
import numpy as np
import pytest

from oracle import potential as pot, step as S
from oracle.systems import Params
from paper_2501_11767_amd import inputs

BETAS = (2e-4, 2e-4, 1e-3, 4e-3)
PQ = dict(eps=0.05, tau=1e-4, mobility=1.0, evap_rate=0.5, viscosity=1.0, alpha=1e-3, betas=BETAS)


def _full(p, n, s, a, Phi):
    """eq. (appPotential) in all four phases, written out independently."""
    P = Phi ** 2 * (3.0 - 2.0 * Phi)
    liq = 3.5 * p * p * n * n + 0.3 * s * s + 0.3 * a * a - 10.0 * s * a
    gas = 3.5 * p * p + 3.5 * n * n + 2.0 * s * s + 0.1 * a * a
    return (1.0 - P) * liq + P * gas


def test_derivatives_match_central_differences():
    g = np.random.default_rng(3)
    p, n, s, Phi = (g.uniform(0.05, 0.4, 20) for _ in range(4))
    q = pot.quaternary(p, n, s, Phi)
    red = lambda p, n, s, Phi: _full(p, n, s, 1.0 - p - n - s, Phi)
    assert np.allclose(q["f"], red(p, n, s, Phi), rtol=1e-14, atol=1e-14)
    e = 1e-6
    for key, d in (("dp", (e, 0, 0, 0)), ("dn", (0, e, 0, 0)), ("ds", (0, 0, e, 0)), ("fv", (0, 0, 0, e))):
        fd = (red(p + d[0], n + d[1], s + d[2], Phi + d[3]) - red(p - d[0], n - d[1], s - d[2], Phi - d[3])) / (2 * e)
        assert np.abs(q[key] - fd).max() < 1e-8, key
    a = 1.0 - p - n - s
    fd = (_full(p, n, s, a + e, Phi) - _full(p, n, s, a - e, Phi)) / (2 * e)
    assert np.abs(q["fa"] - fd).max() < 1e-8


def test_zero_air_reduces_to_the_ternary_density():
    """With phi_s = 1 - phi_p - phi_N (no air) both reductions describe the same
    quartic: equal values, and the ternary derivatives along phi_s = 1 - phi_p -
    phi_N are the quaternary's differences d_i - d_s; the unreduced solvent
    derivative is d_s + f_a."""
    g = np.random.default_rng(4)
    p, n, Phi = g.uniform(0.05, 0.45, 30), g.uniform(0.05, 0.45, 30), g.uniform(0, 1, 30)
    s = 1.0 - p - n
    q = pot.quaternary(p, n, s, Phi)
    t = pot.ternary(p, n, Phi, pot.Quartic())
    assert np.allclose(q["f"], t["f"], rtol=1e-14, atol=1e-15)
    assert np.allclose(q["dp"] - q["ds"], t["dp"], rtol=1e-13, atol=1e-14)
    assert np.allclose(q["dn"] - q["ds"], t["dn"], rtol=1e-13, atol=1e-14)
    assert np.allclose(q["ds"] + q["fa"], t["fs"], rtol=1e-13, atol=1e-14)
    assert np.allclose(q["fv"], t["fv"], rtol=1e-13, atol=1e-14)


def _state(n, prm, seed=5, vel=True):
    ops = S.Operators(n, need_p2=True)
    f = inputs.initial_state(n, "quaternary", 0.33, seed)
    if not vel:
        f["vel"] = np.zeros_like(f["vel"])
    return ops, S.initial_state(ops, prm, "quaternary", f)


def test_initial_film_and_air():
    n = 16
    f = inputs.initial_state(n, "quaternary", 0.33, 1)
    air = 1.0 - f["phi"][0] - f["phi"][1] - f["phi"][2]
    film = f["Phi_v"] < 0.5
    assert np.all(np.abs(air[film]) <= 0.03) and np.all(air[~film] == 1.0)
    assert np.all(np.abs(f["phi"][2][film] - 0.34) <= 0.01)


def test_step_conserves_every_phase_and_solves_per_phase_systems():
    """Without convection every CH row block sums to 1^T M (phi^{k+1} - phi^k),
    so each phase's mass and hence the air's is kept; each phase's system
    carries its own beta."""
    n = 16
    prm = Params(**PQ)
    ops, st = _state(n, prm, vel=False)
    out, sysr = S.step(ops, prm, "quaternary", st, return_systems=True)
    for i in range(3):
        m0, m1 = S.mass(ops, st["phi"][i]), S.mass(ops, out["phi"][i])
        assert abs(m1 - m0) <= 1e-12 * max(abs(m0), 1e-3)
    A = sysr["ch_all"]
    assert A[0] is A[1] and A[1] is not A[2]  # beta_p = beta_N != beta_s
    N = n * n
    c22 = [A[i][N:, N:].diagonal()[0] / ops.M.diagonal()[0] for i in range(3)]
    for i in range(3):
        assert abs(c22[i] + prm.tau * prm.gamma / BETAS[i]) < 1e-9 * abs(c22[i])
        x = np.concatenate([out["phi"][i], out["mu"][i]])
        assert np.linalg.norm(A[i] @ x - sysr["ch_rhs"][i]) <= 1e-11 * np.linalg.norm(sysr["ch_rhs"][i])


def test_constant_state_closure():
    """Constant fields: K annihilates them, so the phases stay, mu_i = d_i and
    mu_a = f_a of the quartic at that state."""
    n = 8
    prm = Params(**PQ)
    ops = S.Operators(n, need_p2=True)
    c = (0.2, 0.25, 0.3)
    f = dict(phi=[np.full(n * n, v) for v in c], Phi_v=np.full(n * n, 0.4),
             vel=np.zeros((2, 4 * n * n)), p=np.zeros(n * n))
    st = S.initial_state(ops, prm, "quaternary", f)
    out = S.step(ops, prm, "quaternary", st)
    q = pot.quaternary(*c, 0.4)
    for i, k in enumerate(("dp", "dn", "ds")):
        assert np.abs(out["phi"][i] - c[i]).max() < 1e-13
        assert np.abs(out["mu"][i] - q[k]).max() < 1e-11
    assert np.abs(out["mu_a"] - q["fa"]).max() < 1e-11
    assert np.abs(out["vel"]).max() < 1e-12  # no gradients: no Korteweg force


def test_polymer_and_nfa_are_interchangeable():
    """The quartic is symmetric in phi_p and phi_N and beta_p = beta_N: swapping
    the two input phases swaps the outputs and leaves the rest unchanged."""
    n = 16
    prm = Params(**PQ)
    ops, st = _state(n, prm)
    a = S.step(ops, prm, "quaternary", st)
    sw = dict(st, phi=[st["phi"][1], st["phi"][0], st["phi"][2]], mu=[st["mu"][1], st["mu"][0], st["mu"][2]])
    b = S.step(ops, prm, "quaternary", sw)
    tol = 1e-11
    assert np.abs(a["phi"][0] - b["phi"][1]).max() < tol and np.abs(a["phi"][1] - b["phi"][0]).max() < tol
    assert np.abs(a["mu"][2] - b["mu"][2]).max() < tol * np.abs(a["mu"][2]).max()
    assert np.abs(a["vel"] - b["vel"]).max() < tol * np.abs(a["vel"]).max()
    assert np.abs(a["mu_a"] - b["mu_a"]).max() < tol * np.abs(a["mu_a"]).max()


def test_small_step_decreases_the_energy():
    n = 16
    prm = Params(**dict(PQ, tau=1e-6))
    ops, st = _state(n, prm, vel=False)
    E0 = S.energy_quaternary(ops, prm, *st["phi"], st["Phi_v"])
    out = S.step(ops, prm, "quaternary", st)
    E1 = S.energy_quaternary(ops, prm, *out["phi"], out["Phi_v"])
    assert E1 < E0


def test_per_phase_betas_are_quaternary_only():
    n = 8
    ops = S.Operators(n, need_p2=True)
    prm = Params(**dict(PQ, betas=(1e-3,) * 4))
    st = inputs.initial_state(n, "ternary", 0.3, 2)
    with pytest.raises(ValueError):
        S.initial_state(ops, prm, "ternary", st)
    with pytest.raises(ValueError):
        _, sq = _state(n, Params(**dict(PQ, rho_pure=(1.0, 1.0, 1.0))))
        S.step(ops, Params(**dict(PQ, rho_pure=(1.0, 1.0, 1.0))), "quaternary", sq)
