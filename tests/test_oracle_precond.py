"""Pins of the oracle's preconditioners, multigrid cycle and Krylov reference.

* Matching Schur approximation: for C = 0 the eigenvalues of S~^{-1} S lie in
  [1/2, 1] (the matching argument behind eq. (schurCH)); with the factor
  printed the second time (beta squared) they do not.
* The V-cycle is a convergent linear iteration, symmetric for symmetric
  operators; Galerkin coarse operators of M and K are the rediscretised ones
  (nested spaces).
* Flexible GMRES reaches the direct solution and, after N steps on an N x N
  system, is exact.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import krylov, multigrid as mg, precond as PC, solvers, step as S, systems
from oracle.systems import Params
from paper_2501_11767_amd import inputs

PARAMS = [(1e-3, 1.0, 0.02), (1e-2, 10.0, 0.005), (1e-5, 0.1, 0.05), (1e-4, 1.0, 0.005)]


@pytest.mark.parametrize("n", [8, 16])
@pytest.mark.parametrize("tau,gamma,eps", PARAMS)
def test_matching_schur_spectrum(n, tau, gamma, eps):
    ops = S.Operators(n)
    prm = Params(eps=eps, tau=tau, mobility=gamma)
    Sx = PC.schur_exact(ops.M, ops.K, prm)
    St = PC.schur_matching(ops.M, ops.K, prm)
    ev = sla.eigvals(Sx, St)
    assert np.abs(ev.imag).max() < 1e-8
    assert ev.real.min() >= 0.5 - 1e-9 and ev.real.max() <= 1.0 + 1e-9


def test_matching_factor_with_beta_squared_breaks_the_bound():
    n = 8
    ops = S.Operators(n)
    prm = Params(eps=0.02, tau=1e-3, mobility=1.0)
    t, g, b = prm.tau, prm.gamma, prm.beta
    X = (t * g * ops.K + np.sqrt(t * g / b ** 2) * ops.M).toarray()
    St = X @ np.linalg.solve(ops.M.toarray(), X)
    ev = sla.eigvals(PC.schur_exact(ops.M, ops.K, prm), St).real
    assert ev.min() < 0.5 - 1e-3


def test_prolongation_interpolates_linear_functions():
    # P1 interpolation reproduces a function linear in x on the fine mesh
    # away from the periodic seam.
    nf = 16
    P = mg.prolongation(nf).toarray()
    nc = nf // 2
    assert np.allclose(P.sum(axis=1), 1.0)
    c = np.arange(nc * nc) % nc  # coarse x index
    fx = P @ c.astype(float)
    fi = np.arange(nf * nf) % nf
    inside = fi < nf - 1
    assert np.allclose(fx[inside], fi[inside] / 2.0)


def test_galerkin_equals_rediscretisation():
    n = 16
    fine, coarse = S.Operators(n), S.Operators(n // 2)
    P = mg.prolongation(n)
    for Af, Ac in ((fine.M, coarse.M), (fine.K, coarse.K)):
        G = (P.T @ Af @ P).toarray()
        assert np.allclose(G, Ac.toarray(), atol=1e-14)


@pytest.mark.parametrize("tau", [1e-5, 1e-2])
def test_vcycle_converges_and_is_symmetric(tau):
    n = 32
    ops = S.Operators(n)
    prm = Params(eps=0.01, tau=tau, mobility=1.0)
    X = PC.matching_factor(ops.M, ops.K, prm)
    a, b = np.sqrt(prm.tau * prm.gamma / prm.beta), prm.tau * prm.gamma
    H = mg.Hierarchy(X, n, a=a, b=b, rho_cut=0.0)
    assert H.sizes == [32, 16, 8, 4]
    N = n * n
    # symmetric: <x, B y> = <y, B x> for the cycle operator B
    g = np.random.default_rng(1)
    x, y = g.standard_normal(N), g.standard_normal(N)
    assert abs(x @ mg.vcycle(H, y) - y @ mg.vcycle(H, x)) < 1e-10 * abs(x @ mg.vcycle(H, x))
    e = g.standard_normal(N)
    e0 = np.linalg.norm(e)
    for _ in range(5):
        e = e - mg.vcycle(H, X @ e)
    assert (np.linalg.norm(e) / e0) ** (1 / 5) < 0.3


def test_chebyshev_matches_the_chebyshev_polynomial():
    # For A = diag(lam), D = I, x0 = 0: the error after k steps is
    # T_k((theta - lam)/delta) / T_k(theta/delta) times the initial error.
    lo, hi, k = 0.3, 2.0, 5
    lam = np.linspace(0.05, 2.0, 40)
    A = sp.diags(lam).tocsr()
    x = mg.chebyshev(A, np.ones(40), np.ones(40), np.zeros(40), lo, hi, k)
    e = x - 1.0 / lam
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    T = lambda t: np.cosh(k * np.arccosh(t)) if t >= 1 else np.cos(k * np.arccos(np.clip(t, -1, 1)))
    ref = np.array([T((theta - l) / delta) for l in lam]) / T(theta / delta) * (-1.0 / lam)
    assert np.allclose(e, ref, rtol=1e-10, atol=1e-12)


def test_level_cut_rule():
    sizes = mg.level_sizes(1024)
    assert sizes == [1024, 512, 256, 128, 64, 32, 16, 8, 4]
    assert mg.cut_level(sizes, 1.0, 0.0) == 0          # pure mass: fine level only
    # rho_l = 8 b n_l^2 / a <= 0.25 first at n_l = 16 for b/a = 1e-4 / 2
    assert mg.cut_level(sizes, 2.0, 1e-4) == 6
    assert mg.cut_level(sizes, 1.0, 1.0) == len(sizes) - 1


def test_fgmres_reaches_direct_solution_with_block_preconditioner():
    n = 16
    ops = S.Operators(n)
    prm = Params(eps=0.05, tau=1e-3, mobility=1.0)
    f = inputs.initial_state(n, "ch", 0.5, 3)
    f["vel"] = inputs.stream_velocity(n, 4, amp=0.05)
    st = S.initial_state(ops, prm, "ch", f)
    out, sysr = S.step(ops, prm, "ch", st, "splu", return_systems=True)
    A, b = sysr["ch"], sysr["ch_rhs"][0]
    from oracle import fem
    C = fem.p1_convection(ops.mesh, f["vel"])
    for inner in ("exact", "mg"):
        P = PC.CHPreconditioner(ops.M, ops.K, C, prm, n, inner=inner)
        x, its, hist = krylov.fgmres(A, b, prec=P.apply, rtol=1e-12, restart=40)
        xs = np.concatenate([out["phi"][0], out["mu"][0]])
        assert np.linalg.norm(x - xs) < 1e-9 * np.linalg.norm(xs)
        assert its < 120


def test_fgmres_is_exact_after_n_steps():
    g = np.random.default_rng(2)
    N = 12
    A = g.standard_normal((N, N)) + N * np.eye(N)
    b = g.standard_normal(N)
    x, its, _ = krylov.fgmres(A, b, fixed_iters=N)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10)
