"""Discrete adjoint of the ternary step (differentiation form), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The scheme of section "Spatial & temporal discretization" maps the state
s^k = (phi_p, phi_N, mu_p, mu_N, mu_s, Phi_v, v, p)^k to s^{k+1} through the
linear systems of section "Iterative solvers and preconditioning" (two CH
solves with the same matrix, the AC solve, the Oseen solve) and the closure of
the eliminated phase.  For a loss L(s^N) the reverse sweep is

    lambda^N = dL/ds^N,   lambda^k = (ds^{k+1}/ds^k)^T lambda^{k+1},
    dL/dtheta = sum_k (ds^{k+1}/dtheta)^T lambda^{k+1},

with theta = (eps, mobility, evaporation rate) entering through beta = eps^2,
gamma = mobility, gamma_v = evaporation rate, delta_v = gamma_v eps^2 and the
Korteweg coefficients beta_i = beta_v = eps^2.  Each linear solve A x = b(s^k)
with A = A(s^k) contributes through eta = A^{-T} lambda_x:

    lambda_{s^k} += (db/ds^k)^T eta - (d(A x)/ds^k)^T eta,
    dL/dtheta    += eta^T (db/dtheta - (dA/dtheta) x).

The pressure never enters a later step, so its adjoint is zero.  The initial
state (including mu^0) is data, independent of theta.

Building blocks: Hessian entries of the ternary density (hand derivatives of
the functions in ``potential``), and vector-Jacobian products of the P1
convection form in v, of the P2 convection form in its convecting field, of
the Korteweg load in the phase gradients, and of the elementwise gradient.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fem, potential as pot, solvers, step as S, systems
from .systems import Params


# ---------------------------------------------------------------- potentials


def hess_ter(pp, pn, Phi, prm: Params | None = None):
    """Second derivatives of the reduced ternary density (nodal), from
    potential.ternary: 'pp', 'pn', 'nn' (d f_i' / d phi_j), 'pP', 'nP'
    (d f_i' / d Phi), 'vp', 'vn', 'vP' (d f_v' / d phi_p, phi_N, Phi) with
    f_v' = df/dPhi, and 'sp', 'sn', 'sP' (d f_s' / d phi_p, d phi_N, d Phi) for
    the closure density f_s'."""
    t = S.ternary_potential(prm if prm is not None else Params(eps=1.0, tau=1.0), pp, pn, Phi)
    return {"pp": t["hpp"], "nn": t["hnn"], "pn": t["hpn"], "pP": t["hpP"], "nP": t["hnP"],
            "vp": t["hpP"], "vn": t["hnP"], "vP": t["hvP"], "sp": t["hsp"], "sn": t["hsn"],
            "sP": t["hsP"], "dp": t["dp"], "dn": t["dn"], "fv": t["fv"]}


# ---------------------------------------------------------------- form VJPs


def p1_conv_vjp(m: fem.Mesh, eta, x):
    """Gradient in the P2 convecting field v (2, 4N) of eta^T C(v) x, where
    C_ij = int (v . grad phi_j) phi_i (the form of ``fem.p1_convection``)."""
    phi = fem.p1_basis(fem.QP)
    psi = fem.p2_basis(fem.QP)
    eta_q = np.einsum("qa,ea->eq", phi, eta[m.tri])
    gx = fem.p1_grad(m, x)
    ge = np.einsum("e,q,eq,qk,ed->edk", m.area, fem.QW, eta_q, psi, gx)
    out = np.zeros((2, 4 * m.nv))
    for d in range(2):
        np.add.at(out[d], m.tri2.ravel(), ge[:, d, :].ravel())
    return out


def p2_conv_vjp(m: fem.Mesh, xi, u):
    """Gradients of sum_c xi_c^T J(w, w_c) u_c, J the scalar P2 convection of
    ``fem.p2_convection``: in the P2 field w (2, 4N) and in the
    elementwise-constant part w_c (ne, 2)."""
    psi = fem.p2_basis(fem.QP)
    G = fem._p2_grads(m)  # (ne, nq, 6, 2)
    # s[e, q, d] = sum_c xi_c(q) d_d u_c(q)
    s = np.zeros((m.ne, len(fem.QW), 2))
    for c in range(2):
        xq = np.einsum("qk,ek->eq", psi, xi[c][m.tri2])
        gu = np.einsum("eqkd,ek->eqd", G, u[c][m.tri2])
        s += xq[..., None] * gu
    gw_e = np.einsum("e,q,qk,eqd->edk", m.area, fem.QW, psi, s)
    gw = np.zeros((2, 4 * m.nv))
    for d in range(2):
        np.add.at(gw[d], m.tri2.ravel(), gw_e[:, d, :].ravel())
    gc = np.einsum("e,q,eqd->ed", m.area, fem.QW, s)
    return gw, gc


def grad_T(m: fem.Mesh, ge):
    """Transpose of ``fem.p1_grad``: b_n = sum_e ge_e . grad phi_n on e."""
    be = np.einsum("ed,ead->ea", ge, m.grad)
    b = np.zeros(m.nv)
    np.add.at(b, m.tri.ravel(), be.ravel())
    return b


def korteweg_vjp(m: fem.Mesh, xi, fields, betas):
    """Gradients of xi^T F(u_1, ..., u_r) in each P1 field u_i, F the load of
    ``fem.korteweg_load`` with G = sum_i beta_i grad u_i (x) grad u_i."""
    Gp = fem._p2_grads(m)
    intgrad = np.einsum("e,q,eqkd->ekd", m.area, fem.QW, Gp)
    N2 = 4 * m.nv
    Y = np.stack([np.einsum("ek,ekd->ed", xi[c * N2:(c + 1) * N2][m.tri2], intgrad)
                  for c in range(2)], axis=1)  # Y[e, c, d]
    Ys = Y + np.transpose(Y, (0, 2, 1))
    out = []
    for u, b in zip(fields, betas):
        g = fem.p1_grad(m, u)
        out.append(grad_T(m, b * np.einsum("ecd,ed->ec", Ys, g)))
    return out


# ---------------------------------------------------------------- one step


def zero_adjoint(N):
    """Zero adjoint state for N P1 nodes (4N P2 ids per velocity component)."""
    return dict(phi=[np.zeros(N), np.zeros(N)], mu=[np.zeros(N), np.zeros(N)], mu_s=np.zeros(N),
                Phi_v=np.zeros(N), vel=np.zeros((2, 4 * N)), p=np.zeros(N))


def next_state(out):
    return dict(phi=out["phi"], mu=out["mu"], mu_s=out["mu_s"], Phi_v=out["Phi_v"],
                vel=out["vel"], p=out["p"])


def step_vjp(ops: S.Operators, prm: Params, st, st1, lam1):
    """Adjoint of one ternary step: (lambda^k, dL/dtheta contribution) from the
    state s^k, the state s^{k+1} it produced and lambda^{k+1}."""
    if prm.rho_pure is not None or prm.picard > 1:
        raise NotImplementedError("the reverse step covers the linear scheme with constant density")
    n, N = ops.n, ops.N
    m, M, K = ops.mesh, ops.M, ops.K
    eps, tau, gam, gv = prm.eps, prm.tau, prm.gamma, prm.gamma_v
    beta = prm.beta
    c = tau * gam / beta
    pp, pn, Phi = st["phi"][0], st["phi"][1], st["Phi_v"]
    H = hess_ter(pp, pn, Phi, prm)
    fps = (H["dp"], H["dn"])
    fv = H["fv"]
    lam = zero_adjoint(N)
    dth = np.zeros(3)
    C = fem.p1_convection(m, st["vel"])

    # closure mu_s^{k+1} = f_s'(phi_s^k, Phi^k) + beta M^{-1} K phi_s^{k+1}
    nu_s = lam1["mu_s"]
    q = beta * (K @ ops.mass_solve(nu_s))
    lam["phi"][0] += H["sp"] * nu_s
    lam["phi"][1] += H["sn"] * nu_s
    lam["Phi_v"] += H["sP"] * nu_s
    ps1 = 1.0 - st1["phi"][0] - st1["phi"][1]
    dth[0] += nu_s @ (2.0 * eps * ops.mass_solve(K @ ps1))

    # Cahn-Hilliard blocks (one matrix, two right-hand sides)
    Ach = systems.ch_matrix(M, K, C, prm)
    lu = spla.splu(Ach.T.tocsc())
    g = []
    for i in range(2):
        eta = lu.solve(np.concatenate([lam1["phi"][i] - q, lam1["mu"][i]]))
        e1, e2 = eta[:N], eta[N:]
        x1, x2 = st1["phi"][i], st1["mu"][i]
        lam["phi"][i] += M @ e1
        g.append(-c * (M @ e2))
        lam["vel"] -= tau * p1_conv_vjp(m, e1, x1)
        # db/dgamma = [0; -(tau/beta) M f'], dA/dgamma = [[0, tau K], [tau K, -(tau/beta) M]]
        dth[1] += (-(tau / beta) * (e2 @ (M @ fps[i]))
                   - (e1 @ (tau * (K @ x2)) + e2 @ (tau * (K @ x1) - (tau / beta) * (M @ x2))))
        # beta = eps^2: db2/deps = (2 tau gam / eps^3) M f', dA22/deps = (2 tau gam / eps^3) M
        dth[0] += (2.0 * tau * gam / eps ** 3) * (e2 @ (M @ (fps[i] - x2)))
    lam["phi"][0] += H["pp"] * g[0] + H["pn"] * g[1]
    lam["phi"][1] += H["pn"] * g[0] + H["nn"] * g[1]
    lam["Phi_v"] += H["pP"] * g[0] + H["nP"] * g[1]

    # Allen-Cahn: (M + tau delta_v K + tau C) Phi^{k+1} = M Phi^k - tau gamma_v M f_v'
    Aac = systems.ac_matrix(M, K, C, prm)
    zeta = spla.splu(Aac.T.tocsc()).solve(lam1["Phi_v"])
    Phi1 = st1["Phi_v"]
    lam["Phi_v"] += M @ zeta
    gvv = -tau * gv * (M @ zeta)
    lam["phi"][0] += H["vp"] * gvv
    lam["phi"][1] += H["vn"] * gvv
    lam["Phi_v"] += H["vP"] * gvv
    lam["vel"] -= tau * p1_conv_vjp(m, zeta, Phi1)
    dth[2] += zeta @ (-tau * (M @ fv) - tau * eps ** 2 * (K @ Phi1))
    dth[0] += -(zeta @ (2.0 * tau * gv * eps * (K @ Phi1)))

    # Oseen: A(w^k) [v; p] = (rho/tau) M v^k + F(phi^k, Phi^k), mean-zero p
    ps_k = 1.0 - pp - pn
    mu_grads = [fem.p1_grad(m, u) for u in (st["mu"][0], st["mu"][1], st["mu_s"])]
    w_const = -prm.alpha * (mu_grads[0] + mu_grads[1] + mu_grads[2])
    J = fem.p2_convection(m, prm.rho * st["vel"], w_const)
    Avel = systems.oseen_velocity_block(ops.Mv, J, ops.Ksym(prm.viscosity), prm)
    rhs_v = np.concatenate([lam1["vel"][0], lam1["vel"][1]])
    # closed square: the step holds the no-slip unknowns at zero, so the
    # adjoint solve leaves them out (their entries of lambda^{k+1} act on nothing)
    xi, _, _ = solvers.bordered_oseen_solve(Avel.T.tocsr(), ops.B, M, rhs_v, fixed=ops.vfixed)
    N2 = 4 * N
    xi2 = np.stack([xi[:N2], xi[N2:]])
    u1 = st1["vel"]
    lam["vel"] += (prm.rho / prm.tau) * np.stack([ops.Mv @ xi2[0], ops.Mv @ xi2[1]])
    gw, gc = p2_conv_vjp(m, xi2, u1)
    lam["vel"] -= prm.rho * gw
    gmu = grad_T(m, prm.alpha * gc)
    lam["mu"][0] += gmu
    lam["mu"][1] += gmu
    lam["mu_s"] += gmu
    betas = [beta, beta, beta, prm.beta_v]
    kv = korteweg_vjp(m, xi, [pp, pn, ps_k, Phi], betas)
    lam["phi"][0] += kv[0] - kv[2]
    lam["phi"][1] += kv[1] - kv[2]
    lam["Phi_v"] += kv[3]
    grads = [fem.p1_grad(m, u) for u in (pp, pn, ps_k, Phi)]
    F = fem.korteweg_load(m, grads, betas)
    dth[0] += (2.0 / eps) * (xi @ F)
    return lam, dth


# ---------------------------------------------------------------- rollouts


def rollout(ops: S.Operators, prm: Params, st0, steps: int, how: str = "splu"):
    """States s^0 .. s^steps of the ternary scheme."""
    states = [st0]
    for _ in range(steps):
        states.append(next_state(S.step(ops, prm, "ternary", states[-1], how)))
    return states


def loss(ops: S.Operators, st, target):
    """L = 1/2 sum_{i in p, N} (phi_i - t_i)^T M (phi_i - t_i)."""
    return 0.5 * sum(float((st["phi"][i] - target[i]) @ (ops.M @ (st["phi"][i] - target[i])))
                     for i in range(2))


def gradient(ops: S.Operators, prm: Params, st0, target, steps: int):
    """(L, dL/d(eps, mobility, evaporation rate)) by the reverse sweep."""
    states = rollout(ops, prm, st0, steps)
    L = loss(ops, states[-1], target)
    lam = zero_adjoint(ops.N)
    for i in range(2):
        lam["phi"][i] = ops.M @ (states[-1]["phi"][i] - target[i])
    grad = np.zeros(3)
    for k in range(steps - 1, -1, -1):
        lam, d = step_vjp(ops, prm, states[k], states[k + 1], lam)
        grad += d
    return L, grad
