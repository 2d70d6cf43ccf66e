"""Pins of oracle functions that the step and adjoint tests use but do not fix
on their own: the Korteweg load, the symmetric-gradient viscous form with a
non-solenoidal field, convection by a non-constant field (P1 and P2), the
pressure convection-diffusion Schur approximation, and the P2 multigrid
level's spectral bound and P1 -> P2 transfer.

Each pin is chosen so that a plausible mistake (a dropped term, a sign, a
factor, a transposed contraction) fails it; the mistakes are named next to
the assertions.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fem, multigrid as mg, precond as PC, systems
from oracle.systems import Params
from paper_2501_11767_amd import inputs

TP = 2.0 * np.pi


def _p1(n, f):
    xy = inputs.vertex_coords(n)
    return f(xy[:, 0], xy[:, 1])


def _p2(n, f):
    xy = inputs.p2_coords(n)
    return f(xy[:, 0], xy[:, 1])


# ------------------------------------------------------------------ Korteweg load
# Momentum equation of the model: the capillary force is -sum_i beta_i
# div(grad phi_i (x) grad phi_i); its weak form on the periodic box is
# int G : grad zeta with G = sum_i beta_i grad phi_i (x) grad phi_i.

def _phi_and_force(beta):
    phi = lambda x, y: np.sin(TP * x) * np.cos(2 * TP * y) + 0.3 * np.cos(TP * (x + y))
    px = lambda x, y: TP * np.cos(TP * x) * np.cos(2 * TP * y) - 0.3 * TP * np.sin(TP * (x + y))
    py = lambda x, y: -2 * TP * np.sin(TP * x) * np.sin(2 * TP * y) - 0.3 * TP * np.sin(TP * (x + y))
    pxx = lambda x, y: -TP ** 2 * np.sin(TP * x) * np.cos(2 * TP * y) - 0.3 * TP ** 2 * np.cos(TP * (x + y))
    pyy = lambda x, y: -4 * TP ** 2 * np.sin(TP * x) * np.cos(2 * TP * y) - 0.3 * TP ** 2 * np.cos(TP * (x + y))
    pxy = lambda x, y: -2 * TP ** 2 * np.cos(TP * x) * np.sin(2 * TP * y) - 0.3 * TP ** 2 * np.cos(TP * (x + y))
    # (div G)_c = sum_d d_d(d_c phi d_d phi) = sum_d d_cd phi d_d phi + d_c phi lap phi
    fx = lambda x, y: -beta * (pxx(x, y) * px(x, y) + pxy(x, y) * py(x, y)
                               + px(x, y) * (pxx(x, y) + pyy(x, y)))
    fy = lambda x, y: -beta * (pxy(x, y) * px(x, y) + pyy(x, y) * py(x, y)
                               + py(x, y) * (pxx(x, y) + pyy(x, y)))
    return phi, fx, fy


def test_korteweg_load_consistent_with_minus_div_G():
    """For smooth phi the load tested against a smooth field converges to
    int -div G . zeta at second order.  (The load vector itself is not
    pointwise consistent: the elementwise P1 gradients carry an O(h) error
    that alternates between the two triangles of a cell, so the pairing with
    a smooth field is the consistent quantity.)  A sign error gives a
    relative error of 2, a lost or doubled factor 1/2 or 1."""
    beta = 0.7
    phi, fx, fy = _phi_and_force(beta)
    errs = []
    for n in (16, 32, 64):
        m = fem.Mesh(n)
        F = fem.korteweg_load(m, [fem.p1_grad(m, _p1(n, phi))], [beta])
        R = fem.p2_load_vec(m, fx, fy)
        z = np.concatenate([_p2(n, fx), _p2(n, fy)])
        errs.append(abs(z @ F - z @ R) / abs(z @ R))
    assert errs[-1] < 0.02, errs
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.6, errs


def _element_boundary_load(m, grads, betas):
    """int_T G : grad psi_k by the divergence theorem, G constant on T:
    int_T grad psi_k = sum over the edges e of n_e int_e psi_k, with the P2
    edge integrals L/6 at the edge's end vertices and 2L/3 at its midpoint.
    Independent of the basis gradients used by the assembly."""
    G = np.zeros((m.ne, 2, 2))
    for g, b in zip(grads, betas):
        G += b * np.einsum("ec,ed->ecd", g, g)
    # local P2 nodes: vertices 0..2, edge nodes 3 = (1,2), 4 = (0,2), 5 = (0,1)
    edges = [(1, 2, 3), (0, 2, 4), (0, 1, 5)]
    igrad = np.zeros((m.ne, 6, 2))
    centroid = m.xy.mean(axis=1)
    for a, b, mid in edges:
        t = m.xy[:, b, :] - m.xy[:, a, :]
        nrm = np.stack([t[:, 1], -t[:, 0]], axis=1)  # |nrm| = edge length L
        mpt = 0.5 * (m.xy[:, a, :] + m.xy[:, b, :])
        out = np.sign(np.einsum("ed,ed->e", nrm, mpt - centroid))
        nL = nrm * out[:, None]  # outward normal times L
        igrad[:, a, :] += nL / 6.0
        igrad[:, b, :] += nL / 6.0
        igrad[:, mid, :] += 2.0 * nL / 3.0
    out = []
    for c in range(2):
        be = np.einsum("ed,ekd->ek", G[:, c, :], igrad)
        b = np.zeros(4 * m.nv)
        np.add.at(b, m.tri2.ravel(), be.ravel())
        out.append(b)
    return np.concatenate(out)


@pytest.mark.parametrize("n", [4, 8])
def test_korteweg_load_equals_boundary_integral_form(n):
    """For P1 fields (gradients constant per element) the load is exact; the
    assembly must equal the element boundary-integral form.  Two fields with
    different coefficients, so a wrong contraction index (G_dc d_d psi vs
    the diagonal of G), a missing field or a swapped coefficient fails."""
    m = fem.Mesh(n)
    rng = np.random.default_rng(11)
    u1, u2 = rng.standard_normal(n * n), rng.standard_normal(n * n)
    grads = [fem.p1_grad(m, u1), fem.p1_grad(m, u2)]
    betas = [0.3, 1.7]
    F = fem.korteweg_load(m, grads, betas)
    R = _element_boundary_load(m, grads, betas)
    assert np.abs(F - R).max() <= 1e-13 * np.abs(R).max()
    # the contraction pairs G's second index with the test gradient; with
    # only the diagonal of G (a plausible slip) the two forms disagree
    Gd = [g * np.array([1.0, 0.0]) for g in grads]
    assert np.abs(fem.korteweg_load(m, Gd, betas) - R).max() > 1e-3 * np.abs(R).max()


# ------------------------------------------------------------------ viscous form


def test_sym_stiffness_on_a_gradient_field():
    """u = grad g is not solenoidal: 2 eta div sym grad u = eta (lap u +
    grad div u) = 2 eta grad lap g.  K_sym u_h must converge to the load of
    -2 eta grad lap g at second order; dropping the cross term (lap u alone,
    the solenoidal case) gives half of it, a missing factor 2 likewise."""
    eta = 1.3
    gx = lambda x, y: TP * np.cos(TP * x) * np.sin(2 * TP * y) - 0.5 * TP * np.sin(TP * x)
    gy = lambda x, y: 2 * TP * np.sin(TP * x) * np.cos(2 * TP * y)
    # g = sin(2 pi x) sin(4 pi y) + 0.5 cos(2 pi x): lap g = -5 (2pi)^2 sin sin - 0.5 (2pi)^2 cos
    lx = lambda x, y: -5 * TP ** 3 * np.cos(TP * x) * np.sin(2 * TP * y) + 0.5 * TP ** 3 * np.sin(TP * x)
    ly = lambda x, y: -10 * TP ** 3 * np.sin(TP * x) * np.cos(2 * TP * y)
    errs = []
    for n in (8, 16, 32):
        m = fem.Mesh(n)
        u = np.concatenate([_p2(n, gx), _p2(n, gy)])
        R = fem.p2_load_vec(m, lambda x, y: -2 * eta * lx(x, y), lambda x, y: -2 * eta * ly(x, y))
        errs.append(np.linalg.norm(fem.p2_sym_stiffness(m, eta) @ u - R) / np.linalg.norm(R))
    assert errs[-1] < 0.01, errs
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.7, errs


def test_sym_stiffness_cross_term_equals_grad_div_on_the_torus():
    """The cross term int d_c psi_i d_e psi_j and its transposed variant
    int d_e psi_i d_c psi_j (the grad-div form int div u div zeta) are the
    same matrix on a periodic mesh: int d_d u_c d_c z_d = int div u div z for
    all periodic H1 fields.  So the orientation cannot matter here; it does
    with walls.  Checked entry by entry."""
    n, eta = 6, 0.9
    m = fem.Mesh(n)
    G = fem._p2_grads(m)
    N2 = 4 * n * n
    blocks = [[None, None], [None, None]]
    for e in range(2):
        for c in range(2):
            Ae = np.einsum("e,q,eqa,eqb->eab", m.area, fem.QW, G[..., e], G[..., c])
            if c == e:
                Ae = Ae + np.einsum("e,q,eqad,eqbd->eab", m.area, fem.QW, G, G)
            blocks[e][c] = fem._scatter(m.tri2, m.tri2, eta * Ae, (N2, N2))
    Kv = sp.bmat(blocks, format="csr")
    K = fem.p2_sym_stiffness(m, eta)
    assert abs(Kv - K).max() <= 1e-14 * abs(K).max()


# ------------------------------------------------------------------ convection


def _div_free_field():
    # v = (d_y s, -d_x s), s = sin(2 pi x) sin(2 pi y) + 0.3 cos(2 pi (x + 2y))
    vx = lambda x, y: TP * np.sin(TP * x) * np.cos(TP * y) - 0.6 * TP * np.sin(TP * (x + 2 * y))
    vy = lambda x, y: -(TP * np.cos(TP * x) * np.sin(TP * y) - 0.3 * TP * np.sin(TP * (x + 2 * y)))
    return vx, vy


def _scalar():
    ph = lambda x, y: np.cos(TP * x) * np.sin(2 * TP * y) + 0.5 * np.sin(TP * (x - y))
    phx = lambda x, y: -TP * np.sin(TP * x) * np.sin(2 * TP * y) + 0.5 * TP * np.cos(TP * (x - y))
    phy = lambda x, y: 2 * TP * np.cos(TP * x) * np.cos(2 * TP * y) - 0.5 * TP * np.cos(TP * (x - y))
    return ph, phx, phy


def test_p1_convection_with_a_varying_field_second_order():
    """C(v) phi_h against the load of v . grad phi for a non-constant
    divergence-free v given at the P2 nodes: second order.  Transposing C
    (int (v . grad psi_i) phi_j) turns the sign of the result for
    divergence-free v; a velocity component swap or v evaluated at the wrong
    P2 nodes fails the rate."""
    vx, vy = _div_free_field()
    ph, phx, phy = _scalar()
    errs = []
    for n in (8, 16, 32):
        m = fem.Mesh(n)
        C = fem.p1_convection(m, np.stack([_p2(n, vx), _p2(n, vy)]))
        R = fem.p1_load(m, lambda x, y: vx(x, y) * phx(x, y) + vy(x, y) * phy(x, y))
        errs.append(np.linalg.norm(C @ _p1(n, ph) - R) / np.linalg.norm(R))
        if n == 32:
            assert np.linalg.norm(C.T @ _p1(n, ph) + R) / np.linalg.norm(R) < 0.05
            assert np.linalg.norm(C.T @ _p1(n, ph) - R) / np.linalg.norm(R) > 1.5
    assert errs[-1] < 0.02, errs
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.8, errs


def test_p2_convection_with_a_varying_field_second_order():
    """J(w) u_h (scalar P2) against the load of w . grad u for a non-constant
    w, plus an elementwise-constant part w_c (the -alpha grad mu part of the
    Oseen convecting field) given as the P1 gradient of a smooth function."""
    vx, vy = _div_free_field()
    ph, phx, phy = _scalar()
    cx = lambda x, y: np.cos(TP * y)   # a smooth field sampled at the element centroids
    cy = lambda x, y: 0.5 * np.sin(TP * x)
    errs, errs_c = [], []
    for n in (8, 16, 32):
        m = fem.Mesh(n)
        w = np.stack([_p2(n, vx), _p2(n, vy)])
        J = fem.p2_convection(m, w)
        R = fem.p2_load_vec(m, lambda x, y: vx(x, y) * phx(x, y) + vy(x, y) * phy(x, y),
                            lambda x, y: 0 * x)[:4 * n * n]
        errs.append(np.linalg.norm(J @ _p2(n, ph) - R) / np.linalg.norm(R))
        # elementwise-constant part: its values at the element centroids
        cen = m.xy.mean(axis=1)
        wc = np.stack([cx(cen[:, 0], cen[:, 1]), cy(cen[:, 0], cen[:, 1])], axis=1)
        Jc = fem.p2_convection(m, np.zeros_like(w), wc)
        Rc = fem.p2_load_vec(m, lambda x, y: cx(x, y) * phx(x, y) + cy(x, y) * phy(x, y),
                             lambda x, y: 0 * x)[:4 * n * n]
        errs_c.append(np.linalg.norm(Jc @ _p2(n, ph) - Rc) / np.linalg.norm(Rc))
    assert errs[-1] < 0.01 and errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.8, errs
    # a piecewise-constant coefficient is first-order accurate pointwise
    assert errs_c[-1] < 0.05 and errs_c[0] / errs_c[1] > 1.8 and errs_c[1] / errs_c[2] > 1.9, errs_c


# ------------------------------------------------------------------ PCD Schur approximation


def _pcd_spectrum(n, tau, eta, wamp):
    """Eigenvalues of S^{-1} (B A^{-1} B^T) on mean-zero pressures, with S^{-1}
    applied by the oracle's NS preconditioner (exact inner solves)."""
    vx, vy = _div_free_field()
    m = fem.Mesh(n)
    N, N2 = n * n, 4 * n * n
    prm = Params(eps=0.01, tau=tau, viscosity=eta, rho=1.0)
    w = wamp * np.stack([_p2(n, vx), _p2(n, vy)])
    A = systems.oseen_velocity_block(fem.p2_mass(m), fem.p2_convection(m, w),
                                     fem.p2_sym_stiffness(m, eta), prm)
    B = fem.divergence_matrix(m)
    M, K = fem.p1_mass(m), fem.p1_stiffness(m)
    Ap = PC.pcd_matrix(M, K, fem.p1_convection(m, w), prm)
    P = PC.NSPreconditioner(A, M, K, Ap, prm, n, inner="exact")
    S = B.toarray() @ np.linalg.solve(A.toarray(), B.T.toarray())
    T = np.zeros((N, N))
    for k in range(N):
        r = np.zeros(2 * N2 + N)
        r[2 * N2:] = S[:, k]
        T[:, k] = P.apply(r)[2 * N2:]
    Q = np.linalg.qr(np.eye(N) - 1.0 / N)[0][:, :N - 1]  # orthonormal mean-zero basis
    P0 = np.eye(N) - 1.0 / N
    return sla.eigvals(Q.T @ P0 @ T @ Q)


@pytest.mark.parametrize("tau", [1e-5, 5e-4, 1e-2])
def test_pcd_spectrum_bounded_and_mesh_independent(tau):
    """w = 0: the preconditioned Schur complement has real eigenvalues in
    [0.45, 1] at n = 8 and 16 for tau from 1e-5 to 1e-2 (measured range 0.47
    to 0.99).  Dropping eta K_p from A_p puts the smallest eigenvalue near
    0.01 at tau = 1e-2; dropping (rho/tau) M_p puts the largest near 0.01 at
    tau = 1e-5."""
    ev8, ev16 = (_pcd_spectrum(n, tau, 1.0, 0.0) for n in (8, 16))
    for ev in (ev8, ev16):
        assert np.abs(ev.imag).max() < 1e-8
        assert ev.real.min() > 0.45 and ev.real.max() < 1.0 + 1e-9, (ev.real.min(), ev.real.max())
    assert abs(ev8.real.min() - ev16.real.min()) < 0.08
    assert abs(ev8.real.max() - ev16.real.max()) < 0.08


def test_pcd_spectrum_with_convection_stays_in_the_right_half_plane():
    """Strong convection (|w| ~ 50, tau = 1e-2, eta = 0.1): every eigenvalue
    keeps a positive real part at n = 8 and 16 (measured min 0.16).  With the
    convection of A_p taken with the wrong sign the smallest real part is
    below -0.3."""
    for n in (8, 16):
        ev = _pcd_spectrum(n, 1e-2, 0.1, 5.0)
        assert ev.real.min() > 0.1 and ev.real.max() < 1.6, (ev.real.min(), ev.real.max())


# ------------------------------------------------------------------ P2 multigrid level


@pytest.mark.parametrize("n", [8, 16])
def test_p2_velocity_block_spectral_bound(n):
    """lambda_max(D^{-1} A_xx) <= LMAX_P2 for the P2 velocity component block
    A_xx = (rho/tau) M_v + (K_sym)_xx over the workloads' range of rho/tau
    (10 .. 1e7) and eta (0.1 .. 10); measured maximum 2.20.  The P1 bound
    lambda_max(D^{-1}(a M + b K)) <= 2 behind LMAX = 2.1 is checked too."""
    m = fem.Mesh(n)
    Mv = fem.p2_mass(m)
    N2 = 4 * n * n
    worst = 0.0
    for rt in (1e1, 1e3, 1e5, 1e7):
        for eta in (0.1, 1.0, 10.0):
            Axx = (rt * Mv + fem.p2_sym_stiffness(m, eta)[:N2, :N2]).toarray()
            lam = sla.eigvals(Axx / np.diag(Axx)[:, None]).real.max()
            worst = max(worst, lam)
    assert 2.0 < worst <= mg.LMAX_P2, worst
    M, K = fem.p1_mass(m).toarray(), fem.p1_stiffness(m).toarray()
    for a, b in ((1.0, 0.0), (1.0, 1e-4), (1.0, 1e-2), (1e-3, 1.0), (0.0, 1.0)):
        A = a * M + b * K
        lam = sla.eigvals(A / np.diag(A)[:, None]).real.max()
        assert lam <= 2.0 + 1e-12 < mg.LMAX


def test_p2_to_p1_reproduces_linear_fields():
    """The P1 -> P2 transfer of the velocity hierarchy interpolates exactly:
    a field linear in x and y (away from the periodic seam) has its P2 nodal
    values at the edge midpoints, and constants map to constants."""
    n = 16
    P = mg.p2_to_p1(n)
    assert np.allclose(P @ np.ones(n * n), 1.0)
    f = lambda x, y: 0.3 + 2.0 * x - 1.5 * y
    u = P @ _p1(n, f)
    xy2 = inputs.p2_coords(n)
    exact = f(xy2[:, 0], xy2[:, 1])
    # P2 nodes whose edge does not cross the seam (coordinates below 1 - h/2 + ...)
    h = 1.0 / n
    inside = (xy2[:, 0] < 1.0 - h) & (xy2[:, 1] < 1.0 - h)
    assert inside.sum() > 3 * n * n
    assert np.abs(u[inside] - exact[inside]).max() < 1e-13
