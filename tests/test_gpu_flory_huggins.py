"""GPU parity of the ternary model with the Flory-Huggins density (x ln x by
its Taylor-4 polynomial about 1/2) and with the truncated fields of eq.
(truncateCH), through the C-ABI, against the oracle.

Bars as for the fitted quartic: right-hand sides and the closure density
within 1e-13 (rounding order only), the discrete energy within 1e-12, one
FP64 step (rtol 1e-13) within 1e-10 per field but the pressure (its bar
measured from the oracle's own sensitivity, as in test_gpu_ns), one adjoint
step within 1e-9 per field and for dtheta.
"""
import numpy as np
import pytest

from oracle import adjoint as AD, potential as pot, step as S
from oracle.systems import Params
from paper_2501_11767_amd import inputs

pytestmark = pytest.mark.gpu

P = dict(eps=0.04, tau=1e-4, mobility=1.0, evap_rate=0.1, viscosity=1.0, alpha=1e-8, rho=1.0)
CASES = [("fh", False), ("fh", True), ("quartic", True)]


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


def _params(C, kind, truncate, base=P):
    gpu = dict(base, truncate=int(truncate))
    orc = dict(base, truncate=truncate)
    if kind == "fh":
        gpu.update(C.FLORY_HUGGINS)
        orc["potential"] = pot.FloryHuggins()
    return gpu, Params(**orc)


def _state(n, prm, seed=2, mean=0.3, spread=None):
    ops = S.Operators(n, need_p2=True)
    f = inputs.initial_state(n, "ternary", mean, seed)
    if spread is not None:  # push some nodes outside [0, 1] so the truncation acts
        g = np.random.default_rng(seed)
        f["phi"][0] = f["phi"][0] + spread * g.uniform(-1, 1, n * n)
    return ops, S.initial_state(ops, prm, "ternary", f)


@pytest.mark.parametrize("kind,truncate", CASES)
def test_rhs_closure_and_energy(C, kind, truncate):
    import torch
    n = 16
    N = n * n
    gp, prm = _params(C, kind, truncate)
    ops, st = _state(n, prm, spread=0.5 if truncate else None)
    if truncate:
        assert ((st["phi"][0] < 0) | (1 - st["phi"][0] - st["phi"][1] < 0)).any()
    _, sysr = S.step(ops, prm, "ternary", st, "splu", return_systems=True)
    ctx = C.Context(n, "ternary", **gp)
    vel = _t(st["vel"].ravel())
    mus = [_t(st["mu"][0]), _t(st["mu"][1]), _t(st["mu_s"])]
    ctx.assemble(vel, mus)
    f = ctx.fields(phi=[_t(st["phi"][0]), _t(st["phi"][1])], mu=mus, Phi_v=_t(st["Phi_v"]), vel=vel,
                   p=_t(st["p"]))
    rch = torch.zeros(4 * N, dtype=torch.float64, device="cuda")
    rac = torch.zeros(N, dtype=torch.float64, device="cuda")
    rns = torch.zeros(9 * N, dtype=torch.float64, device="cuda")
    ctx.step_rhs(f, rch, rac, rns)
    torch.cuda.synchronize()
    for got, ref in ((_np(rch)[:2 * N], sysr["ch_rhs"][0]), (_np(rch)[2 * N:], sysr["ch_rhs"][1]),
                     (_np(rac), sysr["ac_rhs"]), (_np(rns)[:8 * N], sysr["ns_rhs"])):
        assert _rel(got, ref) < 1e-13 and _maxrel(got, ref) < 1e-12
    pp, pn, Phi = st["phi"][0], st["phi"][1], st["Phi_v"]
    got = ctx.diagnostics(ctx.fields(phi=[_t(pp), _t(pn)], Phi_v=_t(Phi)))
    E = S.energy_ternary(ops, prm, pp, pn, Phi)
    assert abs(got[4] - E) <= 1e-12 * abs(E), (got[4], E)
    ctx.close()


@pytest.mark.parametrize("kind,truncate", CASES)
def test_timestep_matches_oracle(C, kind, truncate):
    import torch
    from test_gpu_ns import _pressure_sensitivity
    n = 16
    gp, prm = _params(C, kind, truncate)
    ops, st = _state(n, prm, spread=0.5 if truncate else None)
    out, sysr = S.step(ops, prm, "ternary", st, "splu", return_systems=True)
    ctx = C.Context(n, "ternary", **gp)
    fld = dict(phi=[_t(st["phi"][0]), _t(st["phi"][1])],
               mu=[_t(st["mu"][0]), _t(st["mu"][1]), _t(st["mu_s"])],
               Phi_v=_t(st["Phi_v"]), vel=_t(st["vel"].ravel()), p=_t(st["p"]))
    f = ctx.fields(**fld)
    print(f"ternary step, {kind} truncate={truncate}", flush=True)
    rc, infos = ctx.timestep(f, f, nsteps=1, opts=C.default_opts(rtol=1e-13, maxiter=400))
    torch.cuda.synchronize()
    assert rc == C.OK and all(i["converged"] for i in infos), infos
    pairs = [(fld["phi"][i], out["phi"][i]) for i in range(2)] + \
            [(fld["mu"][i], out["mu"][i]) for i in range(2)] + \
            [(fld["Phi_v"], out["Phi_v"]), (fld["vel"], out["vel"].ravel()), (fld["mu"][2], out["mu_s"])]
    for got, ref in pairs:
        assert _rel(_np(got), ref) < 1e-10 and _maxrel(_np(got), ref) < 1e-10
    pbar = 10 * _pressure_sensitivity(ops, sysr, out["p"])
    assert _rel(_np(fld["p"]), out["p"]) < pbar, pbar
    ctx.close()


@pytest.mark.parametrize("kind,truncate", [("fh", False), ("fh", True), ("quartic", True)])
def test_adjoint_step_matches_oracle(C, kind, truncate):
    import torch
    from paper_2501_11767_amd import adjoint as A
    n = 16
    N = n * n
    base = dict(eps=0.05, tau=2e-5, mobility=1.3, evap_rate=0.4, viscosity=1.0, alpha=0.1, rho=1.0)
    gp, prm = _params(C, kind, truncate, base)
    ops, st = _state(n, prm, seed=21, spread=0.3 if truncate else None)
    st1 = AD.next_state(S.step(ops, prm, "ternary", st))
    rng = np.random.default_rng(8)
    lam1 = AD.zero_adjoint(n * n)
    for i in range(2):
        lam1["phi"][i] = rng.standard_normal(N)
        lam1["mu"][i] = rng.standard_normal(N)
    lam1["mu_s"] = rng.standard_normal(N)
    lam1["Phi_v"] = rng.standard_normal(N)
    lam1["vel"] = rng.standard_normal((2, 4 * N))
    lam0, dth = AD.step_vjp(ops, prm, st, st1, lam1)
    ctx = C.Context(n, "ternary", **gp)
    tog = lambda s: dict(phi_p=_t(s["phi"][0]), phi_n=_t(s["phi"][1]), mu_p=_t(s["mu"][0]), mu_n=_t(s["mu"][1]),
                         mu_s=_t(s["mu_s"]), Phi=_t(s["Phi_v"]), vel=_t(np.asarray(s["vel"]).ravel()),
                         p=_t(s.get("p", np.zeros(N))))
    g0, g1, gl = tog(st), tog(st1), tog(dict(lam1, p=np.zeros(N)))
    outs = A.empty_state(n)
    opts = C.default_opts(rtol=1e-13, precision=C.F64, maxiter=2000)
    print(f"adjoint step, {kind} truncate={truncate}", flush=True)
    rc, d, info = ctx.timestep_adjoint(A.fields_of(ctx, g0), A.fields_of(ctx, g1), A.fields_of(ctx, gl),
                                       A.fields_of(ctx, outs), opts)
    torch.cuda.synchronize()
    assert rc == C.OK, info
    ref = dict(phi_p=lam0["phi"][0], phi_n=lam0["phi"][1], mu_p=lam0["mu"][0], mu_n=lam0["mu"][1],
               mu_s=lam0["mu_s"], Phi=lam0["Phi_v"], vel=lam0["vel"].ravel())
    for k, r in ref.items():
        assert _rel(_np(outs[k]), r) < 1e-9, (k, _rel(_np(outs[k]), r))
    for j in range(3):
        assert abs(d[j] - dth[j]) <= 1e-9 * abs(dth[j]), (j, d[j], dth[j])
    ctx.close()


def test_flory_huggins_rejected_for_binary_models(C):
    with pytest.raises(C.ChnsError):
        C.Context(16, "ch_ac", eps=0.02, tau=1e-3, **C.FLORY_HUGGINS)
    bad = dict(C.FLORY_HUGGINS, fh_phisat=(0.0, 1e-8, 1e-6))
    with pytest.raises(C.ChnsError):
        C.Context(16, "ternary", eps=0.02, tau=1e-3, **bad)
