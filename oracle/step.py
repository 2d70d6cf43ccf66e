"""One semi-implicit time step by direct solves (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Spatial & temporal discretization" (semi-implicit scheme: linear
terms implicit, potential terms explicit, Navier-Stokes nonlinearity lagged)
and section "Iterative solvers and preconditioning" (the three linear systems).
Reading of the coupling: every coupling term is taken at time level k (v^k in
the convection matrix, phi^k and Phi^k in the potentials and in the Korteweg
force, mu^k and v^k in the Oseen convecting field), so the sub-solves of one
step are independent of each other.

Models:
* ``ch``      one phase, double-well potential, no vapour field.
* ``ch_ac``   one phase plus the vapour field, liquid/gas interpolated potential.
* ``ternary`` polymer and NFA phases (solvent = 1 - phi_p - phi_N), vapour
              field and the Oseen step; the eliminated phase's chemical
              potential is recovered from the second CH equation (the paper's
              air-elimination procedure in section "Numerical results", applied
              to the solvent).
* ``quaternary`` the paper's full system: polymer, NFA and solvent phases with
              the air eliminated (phi_a = 1 - phi_p - phi_N - phi_s), the
              fitted quartic of eq. (appPotential) with its air terms, a
              gradient coefficient per phase, mu_a from eq. (airdisc), the
              vapour field and the Oseen step with all four phases in the
              Korteweg force and the convecting field.
"""
from __future__ import annotations

import numpy as np

from . import fem, potential as pot, solvers, systems
from .systems import Params


class Operators:
    """Mesh plus the step-independent matrices.  box_length: the closed
    square [0, L]^2 (fem.BoxMesh) with no-flux boundaries for the phase and
    vapour fields and no-slip walls for the velocity, instead of the periodic
    unit square."""

    def __init__(self, n: int, need_p2: bool = False, box_length: float | None = None):
        self.n = n
        self.box = box_length is not None
        self.mesh = fem.BoxMesh(n, box_length) if self.box else fem.Mesh(n)
        self.N = self.mesh.nv
        # velocity unknowns held at zero (no-slip walls of the closed square)
        self.vfixed = np.concatenate([self.mesh.p2_fixed()] * 2) if (self.box and need_p2) else None
        self.M = fem.p1_mass(self.mesh)
        self.K = fem.p1_stiffness(self.mesh)
        self.Mv = fem.p2_mass(self.mesh) if need_p2 else None
        self.B = fem.divergence_matrix(self.mesh) if need_p2 else None
        self._Ksym = {}

    def Ksym(self, eta):
        if eta not in self._Ksym:
            self._Ksym[eta] = fem.p2_sym_stiffness(self.mesh, eta)
        return self._Ksym[eta]

    def mass_solve(self, b):
        return solvers.sparse_solve(self.M, b)


class Operators3D:
    """The cube (fem3d.Mesh3, Kuhn tetrahedra; periodic, or closed with
    ``box``: no-flux walls) with the P1 matrices, for the binary models
    without convection."""

    three_d = True
    Mv = B = vfixed = None

    def __init__(self, n: int, length: float = 1.0, box: bool = False):
        from . import fem3d
        self.n = n
        self.box = box
        self.mesh = fem3d.Mesh3(n, length, box)
        self.N = self.mesh.nv
        self.M = fem3d.p1_mass(self.mesh)
        self.K = fem3d.p1_stiffness(self.mesh)

    def mass_solve(self, b):
        return solvers.sparse_solve(self.M, b)


def _solve(A, b, how):
    if how == "dense":
        return solvers.dense_solve(A, b)
    return solvers.sparse_solve(A, b)


def ternary_potential(prm: Params, pp, pn, Phi):
    """The reduced ternary density's nodal terms for the parameter set (see
    potential.ternary)."""
    return pot.ternary(pp, pn, Phi, prm.potential if prm.potential is not None else pot.Quartic(),
                       prm.truncate)


def chemical_potential(ops: Operators, fprime_nodal, phi, beta):
    """mu = M^{-1}(M f' + beta K phi) = f' + beta M^{-1} K phi (second CH equation)."""
    return fprime_nodal + beta * ops.mass_solve(ops.K @ phi)


def initial_state(ops: Operators, prm: Params, model: str, fields: dict):
    """Complete the seeded fields with initial chemical potentials."""
    st = dict(phi=[np.array(f, dtype=np.float64) for f in fields["phi"]],
              Phi_v=None if fields.get("Phi_v") is None else np.array(fields["Phi_v"]),
              vel=None if fields.get("vel") is None else np.array(fields["vel"]),
              p=None if fields.get("p") is None else np.array(fields["p"]))
    if model == "ch":
        fp = [pot.dfdphi_bin(st["phi"][0])]
    elif model == "ch_ac":
        fp = [pot.dfdphi_bin(st["phi"][0], st["Phi_v"])]
    elif model == "quaternary":
        q = pot.quaternary(*st["phi"], st["Phi_v"])
        fp = [q["dp"], q["dn"], q["ds"]]
    else:
        t = ternary_potential(prm, st["phi"][0], st["phi"][1], st["Phi_v"])
        fp = [t["dp"], t["dn"]]
    bs = phase_betas(prm, model)
    st["mu"] = [chemical_potential(ops, f, ph, b) for f, ph, b in zip(fp, st["phi"], bs)]
    if model == "ternary":
        ps = 1.0 - st["phi"][0] - st["phi"][1]
        st["mu_s"] = chemical_potential(ops, t["fs"], ps, prm.beta)
    if model == "quaternary":
        pa = 1.0 - st["phi"][0] - st["phi"][1] - st["phi"][2]
        st["mu_a"] = chemical_potential(ops, q["fa"], pa, bs[3])
    return st


def phase_betas(prm: Params, model: str):
    """Gradient coefficients per phase: (beta_p, beta_N, beta_s, beta_a) for the
    quaternary model, eps^2 for every phase otherwise."""
    if model == "quaternary":
        return [prm.beta_of(i) for i in range(4)]
    if prm.betas is not None:
        raise ValueError("per-phase gradient coefficients belong to the quaternary model")
    return [prm.beta] * 3


def explicit_terms(model, st, prm: Params | None = None):
    """Nodal f'(phi^k) per CH phase and f_v'(Phi^k) for the AC equation."""
    if model == "ch":
        return [pot.dfdphi_bin(st["phi"][0])], None
    if model == "ch_ac":
        return ([pot.dfdphi_bin(st["phi"][0], st["Phi_v"])],
                pot.dfdPhi_bin(st["phi"][0], st["Phi_v"]))
    if model == "quaternary":
        q = pot.quaternary(*st["phi"], st["Phi_v"])
        return [q["dp"], q["dn"], q["ds"]], q["fv"]
    t = ternary_potential(prm if prm is not None else Params(eps=1.0, tau=1.0),
                          st["phi"][0], st["phi"][1], st["Phi_v"])
    return [t["dp"], t["dn"]], t["fv"]


def convecting_field(n: int, prm: Params, rho_k, vel, mesh=None):
    """The P2 field rho v of the Oseen convection (eq. (matrixns)): rho v with
    constant density, else the P2 interpolant of the nodal product of rho^k
    (its P1 interpolant at the P2 nodes) and v.  mesh: the closed square's
    mesh (its padded P2 numbering) instead of the periodic square."""
    if rho_k is None:
        return prm.rho * vel
    if mesh is not None:
        return fem.p2_eval_p1_interp_mesh(mesh, rho_k)[None, :] * vel
    if vel.shape[1] != 4 * n * n:
        raise ValueError("the periodic square's P2 numbering has 4 n^2 nodes")
    return fem.p2_eval_p1_interp(n, rho_k)[None, :] * vel


def step(ops: Operators, prm: Params, model: str, st: dict, how: str = "splu",
         return_systems: bool = False):
    """Advance one step; ``how`` in {"dense", "splu", "fft"} (fft needs v = 0)."""
    n, M, K = ops.n, ops.M, ops.K
    N = ops.N
    mesh = ops.mesh
    vel = st.get("vel")
    C = fem.p1_convection(mesh, vel) if vel is not None else None
    if how == "fft" and (C is not None or ops.box or getattr(ops, "three_d", False)):
        raise ValueError("the Fourier solve needs a convection-free periodic square")
    if getattr(ops, "three_d", False) and (vel is not None or model not in ("ch", "ch_ac")):
        raise ValueError("the cube carries the binary models without convection")
    fps, fv = explicit_terms(model, st, prm)
    out = dict(vel=vel, p=st.get("p"))
    sysrec = {}

    # evaporation flux at the top wall (closed square, one phase: the solvent)
    flux = None
    if prm.top_flux != 0.0:
        if not ops.box or model not in ("ch", "ch_ac"):
            raise ValueError("the top-wall flux belongs to the binary models on the closed square or cube")
        if getattr(ops, "three_d", False):
            from . import fem3d
            ref = n // 2 + (n + 1) * (n // 2) + (n + 1) ** 2 * n  # centre of the top face
            load = fem3d.top_face_load(mesh)
        else:
            ref = n // 2 + (n + 1) * n  # midpoint of the top edge
            load = fem.top_edge_load(mesh)
        j_out = prm.top_flux * (st["phi"][0][ref] - prm.flux_inf)
        flux = j_out * load
        sysrec["j_out"] = j_out

    # Cahn-Hilliard, one solve per phase (the same matrix unless the phases'
    # gradient coefficients differ)
    bs = phase_betas(prm, model)
    mats = {}
    phis, mus = [], []
    for i, (ph, fp) in enumerate(zip(st["phi"], fps)):
        if bs[i] not in mats:
            mats[bs[i]] = systems.ch_matrix(M, K, C, prm, beta=bs[i])
        A_ch = mats[bs[i]]
        sysrec.setdefault("ch_all", []).append(A_ch)
        b = systems.ch_rhs(M, ph, fp, prm, flux, beta=bs[i])
        sysrec.setdefault("ch_rhs", []).append(b)
        if how == "fft":
            if bs[i] != prm.beta:
                raise ValueError("the Fourier solve takes beta = eps^2")
            x1, x2 = solvers.fft_ch_solve(n, prm, b[:N], b[N:])
            x = np.concatenate([x1, x2])
        else:
            x = _solve(A_ch, b, how)
        phis.append(x[:N])
        mus.append(x[N:])
    out["phi"], out["mu"] = phis, mus
    sysrec["ch"] = sysrec["ch_all"][0]

    # Allen-Cahn
    if model in ("ch_ac", "ternary", "quaternary"):
        A_ac = systems.ac_matrix(M, K, C, prm)
        b = systems.ac_rhs(M, st["Phi_v"], fv, prm)
        sysrec["ac"], sysrec["ac_rhs"] = A_ac, b
        out["Phi_v"] = solvers.fft_ac_solve(n, prm, b) if how == "fft" else _solve(A_ac, b, how)
    else:
        out["Phi_v"] = None

    # Oseen step and closure
    if model in ("ternary", "quaternary"):
        if model == "ternary":
            ps_k = 1.0 - st["phi"][0] - st["phi"][1]
            fields = (st["phi"][0], st["phi"][1], ps_k, st["Phi_v"])
            betas = [prm.beta, prm.beta, prm.beta, prm.beta_v]
            mu_all = (st["mu"][0], st["mu"][1], st["mu_s"])
        else:
            if prm.rho_pure is not None:
                raise ValueError("variable density is defined for the ternary model")
            pa_k = 1.0 - st["phi"][0] - st["phi"][1] - st["phi"][2]
            fields = (st["phi"][0], st["phi"][1], st["phi"][2], pa_k, st["Phi_v"])
            betas = bs + [prm.beta_v]
            mu_all = (st["mu"][0], st["mu"][1], st["mu"][2], st["mu_a"])
        grads = [fem.p1_grad(mesh, u) for u in fields]
        w_const = -prm.alpha * sum(fem.p1_grad(mesh, u) for u in mu_all)
        rho_k = systems.density(prm, st["phi"][0], st["phi"][1])
        Mrho = None if rho_k is None else fem.p2_mass_weighted(mesh, rho_k)
        F = fem.korteweg_load(mesh, grads, betas)
        rhs = systems.oseen_rhs(ops.Mv, vel, F, prm, Mrho)
        N2 = 4 * N
        conv = vel  # the velocity the convecting field is formed with
        for m in range(max(1, prm.picard)):
            used = conv
            J = fem.p2_convection(mesh, convecting_field(n, prm, rho_k, conv, mesh if ops.box else None), w_const)
            Avel = systems.oseen_velocity_block(ops.Mv, J, ops.Ksym(prm.viscosity), prm, Mrho)
            v, p, _ = solvers.bordered_oseen_solve(Avel, ops.B, M, rhs, dense=(how == "dense"), fixed=ops.vfixed)
            v = np.stack([v[:N2], v[N2:]])
            change = np.linalg.norm(v - conv) / max(np.linalg.norm(v), 1e-300)
            conv = v
            if m > 0 and change <= prm.picard_tol:
                break
        sysrec["ns_A"], sysrec["ns_rhs"], sysrec["ns_passes"] = Avel, rhs, m + 1
        sysrec["ns_Mrho"], sysrec["ns_conv_vel"], sysrec["ns_w_const"] = Mrho, used, w_const
        out["vel"] = v
        out["p"] = p
        if model == "ternary":
            ps1 = 1.0 - phis[0] - phis[1]
            fs_k = ternary_potential(prm, st["phi"][0], st["phi"][1], st["Phi_v"])["fs"]
            out["mu_s"] = fs_k + prm.beta * ops.mass_solve(K @ ps1)
        else:  # eq. (airdisc) for the air: M mu_a = M f_a^k + beta_a K phi_a^{k+1}
            pa1 = 1.0 - phis[0] - phis[1] - phis[2]
            fa_k = pot.quaternary(*st["phi"], st["Phi_v"])["fa"]
            out["mu_a"] = fa_k + bs[3] * ops.mass_solve(K @ pa1)
    if return_systems:
        return out, sysrec
    return out


def mass(ops: Operators, u):
    """Discrete mass 1^T M u."""
    return float(np.ones(ops.N) @ (ops.M @ u))


def energy_ch(ops: Operators, prm: Params, phi, Phi=None):
    """E_h = beta/2 phi^T K phi + sum_i (M 1)_i f(phi_i) (binary potential)."""
    lump = ops.M @ np.ones(ops.N)
    return 0.5 * prm.beta * phi @ (ops.K @ phi) + lump @ pot.f_bin(phi, Phi)


def energy_ternary(ops: Operators, prm: Params, pp, pn, Phi):
    """Section "Free energy functional" discretised like energy_ch: the
    gradient term beta/2 |grad phi_i|^2 of every phase present (polymer, NFA and
    the eliminated solvent phi_s = 1 - phi_p - phi_N) plus the fitted quartic
    density of the reduced ternary model, nodal with the row sums of M:
    E_h = sum_i beta/2 phi_i^T K phi_i + sum_j (M 1)_j f(phi_p, phi_N, Phi)_j."""
    lump = ops.M @ np.ones(ops.N)
    ps = 1.0 - pp - pn
    grad = sum(u @ (ops.K @ u) for u in (pp, pn, ps))
    return 0.5 * prm.beta * grad + lump @ ternary_potential(prm, pp, pn, Phi)["f"]


def energy_quaternary(ops: Operators, prm: Params, pp, pn, ps, Phi):
    """The discrete free energy of the quaternary model like energy_ternary:
    sum_i beta_i/2 phi_i^T K phi_i over polymer, NFA, solvent and the
    eliminated air, plus sum_j (M 1)_j f(phi_p, phi_N, phi_s, Phi)_j with the
    density of eq. (appPotential)."""
    lump = ops.M @ np.ones(ops.N)
    pa = 1.0 - pp - pn - ps
    bs = phase_betas(prm, "quaternary")
    grad = sum(b * (u @ (ops.K @ u)) for b, u in zip(bs, (pp, pn, ps, pa)))
    return 0.5 * grad + lump @ pot.quaternary(pp, pn, ps, Phi)["f"]
