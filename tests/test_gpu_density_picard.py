"""GPU parity of the variable-density Oseen step and of the Picard passes of
the Oseen solve, through the C-ABI, against the oracle.

Bars as for the constant-density ternary step (test_gpu_ns): operator values
within 1e-12 of the largest entry, right-hand sides within 1e-13, one FP64
step (FGMRES rtol 1e-13 per solve) within 1e-10 for every field but the
pressure, whose bar is ten times the oracle's own sensitivity to rounding-level
perturbations of its system.  With Picard passes the pressure takes the
fields' bar: every pass convects with the previous pass's velocity, so that
velocity's difference enters the next system.
"""
import numpy as np
import pytest

from oracle import fem, precond as PC, step as S, systems
from oracle.systems import Params
from paper_2501_11767_amd import inputs

pytestmark = pytest.mark.gpu

P = dict(eps=0.04, tau=5e-4, mobility=1.0, evap_rate=0.1, viscosity=1.0, alpha=1e-8, rho=1.0)
RHO = (1.3, 0.7, 1.0)
FLOW = dict(P, tau=2e-3, viscosity=0.05)


@pytest.fixture(scope="module")
def C():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_11767_amd import chns
    chns.lib()
    return chns


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _maxrel(a, b):
    return np.abs(np.ravel(a) - np.ravel(b)).max() / max(np.abs(np.ravel(b)).max(), 1e-300)


def _state(n, prm, amp=None, seed=2):
    ops = S.Operators(n, need_p2=True)
    st = S.initial_state(ops, prm, "ternary", inputs.initial_state(n, "ternary", 0.3, seed))
    if amp is not None:
        st["vel"] = inputs.stream_velocity(n, 3, amp=amp)
    return ops, st


def _gpu_params(base, **kw):
    q = dict(base, **kw)
    rp = q.pop("rho_pure", None)
    if rp is not None:
        q.update(var_density=1, rho_pure=rp)
    if "picard" in q:
        q["ns_picard"] = q.pop("picard")
    if "picard_tol" in q:
        q["ns_picard_tol"] = q.pop("picard_tol")
    return q


def _fields(C, ctx, st):
    fld = dict(phi=[_t(st["phi"][0]), _t(st["phi"][1])],
               mu=[_t(st["mu"][0]), _t(st["mu"][1]), _t(st["mu_s"])],
               Phi_v=_t(st["Phi_v"]), vel=_t(np.asarray(st["vel"]).ravel()), p=_t(st["p"]))
    return fld, ctx.fields(**fld)


def _compare_csr(got, ref, tol):
    import scipy.sparse as sp
    rp, col, val, shape = got
    G = sp.csr_matrix((val, col, rp), shape=shape)
    d = (G - sp.csr_matrix(ref)).tocsr()
    scale = np.abs(sp.csr_matrix(ref).data).max()
    assert (np.abs(d.data).max() if d.nnz else 0.0) <= tol * scale


def test_density_operators_and_rhs(C):
    import torch
    n = 16
    N = n * n
    prm = Params(**dict(P, rho_pure=RHO))
    ops, st = _state(n, prm, amp=0.02)
    _, sysr = S.step(ops, prm, "ternary", st, "splu", return_systems=True)
    ctx = C.Context(n, "ternary", **_gpu_params(P, rho_pure=RHO))
    fld, f = _fields(C, ctx, st)
    ctx.set_density(fld["phi"][0], fld["phi"][1])
    ctx.assemble(fld["vel"], fld["mu"])
    _compare_csr(ctx.matrix(C.OP_NS), systems.oseen_matrix(sysr["ns_A"], ops.B), 1e-12)
    # the PCD matrix with the density-weighted pressure mass
    mug = [fem.p1_grad(ops.mesh, u) for u in (st["mu"][0], st["mu"][1], st["mu_s"])]
    wc = -prm.alpha * (mug[0] + mug[1] + mug[2])
    rho = systems.density(prm, st["phi"][0], st["phi"][1])
    Cw = fem.p1_convection(ops.mesh, S.convecting_field(n, prm, rho, st["vel"]), wc)
    Ap = PC.pcd_matrix(ops.M, ops.K, Cw, prm, fem.p1_mass_weighted(ops.mesh, rho))
    _compare_csr(ctx.matrix(C.OP_AP), Ap, 1e-12)
    rch = torch.zeros(4 * N, dtype=torch.float64, device="cuda")
    rac = torch.zeros(N, dtype=torch.float64, device="cuda")
    rns = torch.zeros(9 * N, dtype=torch.float64, device="cuda")
    ctx.step_rhs(f, rch, rac, rns)
    torch.cuda.synchronize()
    got = _np(rns)[:8 * N]
    assert _rel(got, sysr["ns_rhs"]) < 1e-13 and _maxrel(got, sysr["ns_rhs"]) < 1e-12
    ctx.close()


@pytest.mark.parametrize("case", ["density", "picard", "density+picard", "picard-tol"])
def test_step_matches_oracle(C, case):
    import torch
    from test_gpu_ns import _pressure_sensitivity
    n = 16
    kw = {}
    if "density" in case:
        kw["rho_pure"] = RHO
    if case.startswith("picard") or "+picard" in case:
        kw["picard"] = 4 if case != "picard-tol" else 30
    if case == "picard-tol":
        kw["picard_tol"] = 1e-9
    base = FLOW if "picard" in case else P
    prm = Params(**dict(base, **kw))
    ops, st = _state(n, prm, amp=0.05 if "picard" in case else 0.02)
    out, sysr = S.step(ops, prm, "ternary", st, "splu", return_systems=True)
    ctx = C.Context(n, "ternary", **_gpu_params(base, **kw))
    fld, f = _fields(C, ctx, st)
    print(f"ternary step {case}", flush=True)
    rc, infos = ctx.timestep(f, f, nsteps=1, opts=C.default_opts(rtol=1e-13, maxiter=600))
    torch.cuda.synchronize()
    assert rc == C.OK and all(i["converged"] for i in infos), infos
    assert infos[3]["passes"] == sysr.get("ns_passes", 1), (infos[3], sysr.get("ns_passes"))
    pairs = [(fld["phi"][i], out["phi"][i]) for i in range(2)] + \
            [(fld["mu"][i], out["mu"][i]) for i in range(2)] + \
            [(fld["Phi_v"], out["Phi_v"]), (fld["vel"], out["vel"].ravel()), (fld["mu"][2], out["mu_s"])]
    for got, ref in pairs:
        assert _rel(_np(got), ref) < 1e-10 and _maxrel(_np(got), ref) < 1e-10
    pbar = 10 * _pressure_sensitivity(ops, sysr, out["p"])
    if "picard" in case:
        # each pass convects with the previous pass's velocity, whose difference
        # (within the field bar) enters the next matrix: the perturbation of one
        # system does not cover that, so the pressure takes the fields' bar
        pbar = max(pbar, 1e-10)
    assert _rel(_np(fld["p"]), out["p"]) < pbar, pbar
    ctx.close()


def test_picard_reports_and_contracts(C):
    """The Oseen report of a Picard step: passes, the last relative velocity
    change (below the tolerance when it stopped early) and the iterations
    summed over the passes; the CH and AC reports are those of a plain step."""
    import torch
    n = 16
    ops, st = _state(n, Params(**FLOW), amp=0.05)
    ctx = C.Context(n, "ternary", **_gpu_params(FLOW, picard=20, picard_tol=1e-8))
    fld, f = _fields(C, ctx, st)
    one = C.Context(n, "ternary", **FLOW)
    fld1, f1 = _fields(C, one, st)
    rc, infos = ctx.timestep(f, f, 1, C.default_opts(rtol=1e-12, maxiter=600))
    rc1, infos1 = one.timestep(f1, f1, 1, C.default_opts(rtol=1e-12, maxiter=600))
    torch.cuda.synchronize()
    ns, ns1 = infos[3], infos1[3]
    assert 2 <= ns["passes"] < 20 and ns["change"] <= 1e-8, ns
    assert ns1["passes"] == 1 and ns["iters"] > ns1["iters"]
    for i in range(3):  # the CH and AC solves are unchanged
        assert infos[i]["passes"] == 1 and infos[i]["iters"] == infos1[i]["iters"]
    ctx.close()
    one.close()


def test_density_and_picard_are_rejected_where_undefined(C):
    import torch
    with pytest.raises(C.ChnsError):
        C.Context(16, "ch_ac", eps=0.02, tau=1e-3, var_density=1, rho_pure=RHO)
    with pytest.raises(C.ChnsError):
        C.Context(16, "ternary", **_gpu_params(P, rho_pure=(1.0, 0.0, 1.0)))
    with pytest.raises(C.ChnsError):
        C.Context(16, "ternary", **dict(P, ns_picard=101))
    plain = C.Context(16, "ternary", **P)
    z = torch.zeros(256, dtype=torch.float64, device="cuda")
    with pytest.raises(C.ChnsError):
        plain.set_density(z, z)
    plain.close()
    from paper_2501_11767_amd import adjoint as A
    n = 16
    for kw in (dict(rho_pure=RHO), dict(picard=2)):
        ctx = C.Context(n, "ternary", **_gpu_params(P, **kw))
        s = A.empty_state(n)
        with pytest.raises(C.ChnsError) as e:
            ctx.timestep_adjoint(A.fields_of(ctx, s), A.fields_of(ctx, s), A.fields_of(ctx, s),
                                 A.fields_of(ctx, s))
        assert e.value.code == C.EUNSUPPORTED
        ctx.close()
