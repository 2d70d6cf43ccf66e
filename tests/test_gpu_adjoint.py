"""GPU parity of the differentiation form (ternary model), through the C-ABI.

* Transposed operators: <y, A x> on the forward operators equals <A^T y, x> on
  the operators of chns_assemble_transposed, for the CH, AC and Oseen blocks
  (bar 1e-12 relative); likewise the block preconditioners in FP64 with
  mg_pre == mg_post (each V-cycle on A^T is the exact transpose of the one on
  A; the PCD factors reverse), bar 1e-11.
* One adjoint step against the oracle's reverse step from the same s^k,
  s^{k+1} and lambda^{k+1} (the oracle's states, uploaded): transposed
  solves at rtol 1e-13 in FP64, bar 1e-9 relative per field and for dtheta.
* A whole rollout through torch.autograd (checkpoints every 4 steps over 6
  steps, so one segment is partial) against the oracle's gradient with the
  same target: bar 1e-8 relative.
"""
import numpy as np
import pytest

from oracle import adjoint as AD, step as S
from oracle.systems import Params
from paper_2501_11767_amd import inputs

pytestmark = pytest.mark.gpu

BASE = dict(eps=0.05, tau=2e-5, mobility=1.3, evap_rate=0.4, viscosity=1.0, alpha=0.1, rho=1.0)


@pytest.fixture(scope="module")
def mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_11767_amd import adjoint as A, chns as C
    C.lib()
    return C, A


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _oracle_state(n, prm, seed=21, mean=0.3):
    f = inputs.initial_state(n, "ternary", mean, seed)
    ops = S.Operators(n, need_p2=True)
    return ops, S.initial_state(ops, prm, "ternary", f)


def _to_gpu(st):
    return dict(phi_p=_dev(st["phi"][0]), phi_n=_dev(st["phi"][1]), mu_p=_dev(st["mu"][0]),
                mu_n=_dev(st["mu"][1]), mu_s=_dev(st["mu_s"]), Phi=_dev(st["Phi_v"]),
                vel=_dev(np.asarray(st["vel"]).ravel()), p=_dev(st["p"]))


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.mark.parametrize("n", [16, 32])
def test_transposed_operators_and_preconditioners(mods, n):
    import torch
    C, A = mods
    print(f"transposed operators: ternary n={n}", flush=True)
    prm = Params(**BASE)
    _, st = _oracle_state(n, prm)
    g = _to_gpu(st)
    ctx = C.Context(n, "ternary", **BASE)
    mu = [g["mu_p"], g["mu_n"], g["mu_s"]]
    gen = torch.Generator(device="cuda").manual_seed(n)
    N = n * n
    sizes = {C.OP_CH: 2 * N, C.OP_AC: N, C.OP_NS: 9 * N}
    blocks = {C.OP_CH: C.BLOCK_CH, C.OP_AC: C.BLOCK_AC, C.OP_NS: C.BLOCK_NS}
    vecs = {op: (torch.randn(m, dtype=torch.float64, device="cuda", generator=gen),
                 torch.randn(m, dtype=torch.float64, device="cuda", generator=gen)) for op, m in sizes.items()}
    for op, (x, y) in vecs.items():  # mean-zero pressure parts (the preconditioner projects them)
        if op == C.OP_NS:
            x[8 * N:] -= x[8 * N:].mean()
            y[8 * N:] -= y[8 * N:].mean()
    opts = C.default_opts(precision=C.F64)
    fwd, prec = {}, {}
    ctx.assemble(g["vel"], mu)
    for op, (x, y) in vecs.items():
        ax = torch.empty_like(x)
        ctx.spmv(op, x, ax)
        fwd[op] = float(torch.dot(y, ax))
        px = torch.empty_like(x)
        ctx.precond(blocks[op], x, px, opts)
        prec[op] = float(torch.dot(y, px))
    # the transposed products need the transposed operators first
    for op, (x, y) in vecs.items():
        with pytest.raises(C.ChnsError) as e:
            ctx.spmv(op, y, torch.empty_like(y), transpose=True)
        assert e.value.code == C.ESTATE
        with pytest.raises(C.ChnsError) as e:
            ctx.precond(blocks[op], y, torch.empty_like(y), opts, transpose=True)
        assert e.value.code == C.ESTATE
    ctx.assemble_transposed(g["vel"], mu)
    for op, (x, y) in vecs.items():
        with pytest.raises(C.ChnsError) as e:  # and the forward ones the forward operators
            ctx.spmv(op, y, torch.empty_like(y))
        assert e.value.code == C.ESTATE
        aty = torch.empty_like(y)
        ctx.spmv(op, y, aty, transpose=True)
        got = float(torch.dot(aty, x))
        assert abs(got - fwd[op]) <= 1e-12 * abs(fwd[op]), (op, got, fwd[op])
        pty = torch.empty_like(y)
        ctx.precond(blocks[op], y, pty, opts, transpose=True)
        got = float(torch.dot(pty, x))
        assert abs(got - prec[op]) <= 1e-11 * abs(prec[op]), (op, got, prec[op])
    ctx.close()


def test_adjoint_step_matches_oracle(mods):
    import torch
    C, A = mods
    n = 16
    print(f"adjoint step vs oracle: ternary n={n}", flush=True)
    prm = Params(**BASE)
    ops, st = _oracle_state(n, prm)
    st1 = AD.next_state(S.step(ops, prm, "ternary", st))
    rng = np.random.default_rng(8)
    N = n * n
    lam1 = AD.zero_adjoint(n * n)
    for i in range(2):
        lam1["phi"][i] = rng.standard_normal(N)
        lam1["mu"][i] = rng.standard_normal(N)
    lam1["mu_s"] = rng.standard_normal(N)
    lam1["Phi_v"] = rng.standard_normal(N)
    lam1["vel"] = rng.standard_normal((2, 4 * N))
    lam0, dth = AD.step_vjp(ops, prm, st, st1, lam1)

    ctx = C.Context(n, "ternary", **BASE)
    g0, g1, gl = _to_gpu(st), _to_gpu(st1), _to_gpu(dict(lam1, p=np.zeros(N)))
    out = A.empty_state(n)
    opts = C.default_opts(rtol=1e-13, precision=C.F64, maxiter=2000)
    rc, d, info = ctx.timestep_adjoint(A.fields_of(ctx, g0), A.fields_of(ctx, g1), A.fields_of(ctx, gl),
                                       A.fields_of(ctx, out), opts)
    torch.cuda.synchronize()
    assert rc == C.OK, info
    ref = dict(phi_p=lam0["phi"][0], phi_n=lam0["phi"][1], mu_p=lam0["mu"][0], mu_n=lam0["mu"][1],
               mu_s=lam0["mu_s"], Phi=lam0["Phi_v"], vel=lam0["vel"].ravel())
    for k, r in ref.items():
        assert _rel(out[k].cpu().numpy(), r) < 1e-9, (k, _rel(out[k].cpu().numpy(), r))
    assert np.abs(out["p"].cpu().numpy()).max() == 0.0
    for j in range(3):
        assert abs(d[j] - dth[j]) <= 1e-9 * abs(dth[j]), (j, d[j], dth[j])
    # in place (lam_in = lam_out) gives the same result
    rc, d2, _ = ctx.timestep_adjoint(A.fields_of(ctx, g0), A.fields_of(ctx, g1), A.fields_of(ctx, gl),
                                     A.fields_of(ctx, gl), opts)
    torch.cuda.synchronize()
    for k in ref:
        assert _rel(gl[k].cpu().numpy(), out[k].cpu().numpy()) < 1e-12, k
    assert np.allclose(d2, d, rtol=1e-12, atol=0)
    ctx.close()


def test_rollout_gradient_matches_oracle(mods):
    import torch
    C, A = mods
    n, steps = 16, 6
    print(f"rollout gradient vs oracle: ternary n={n}, {steps} steps, checkpoint 4", flush=True)
    ref = dict(BASE, eps=0.05, tau=1e-5, mobility=2.0, evap_rate=0.2, alpha=1e-8)
    th0 = dict(ref, eps=0.045, mobility=1.5, evap_rate=0.15)
    ops, st0 = _oracle_state(n, Params(**ref), seed=33)
    target = AD.rollout(ops, Params(**ref), st0, steps)[-1]["phi"]
    L_ref, g_ref = AD.gradient(ops, Params(**th0), st0, target, steps)

    ctx = C.Context(n, "ternary", **th0)
    theta = torch.tensor([th0["eps"], th0["mobility"], th0["evap_rate"]], dtype=torch.float64,
                         requires_grad=True)
    opts = C.default_opts(rtol=1e-13, precision=C.F64, maxiter=2000)
    php, phn = A.rollout(ctx, theta, _to_gpu(st0), steps, checkpoint=4, opts=opts)
    L = A.loss(ctx, (php, phn), (_dev(target[0]), _dev(target[1])))
    L.backward()
    assert abs(float(L) - L_ref) <= 1e-9 * L_ref
    got = theta.grad.numpy()
    for j in range(3):
        assert abs(got[j] - g_ref[j]) <= 1e-8 * abs(g_ref[j]), (j, got[j], g_ref[j])
    ctx.close()


def test_adjoint_rejects_binary_and_missing_fields(mods):
    import torch
    C, A = mods
    ctx = C.Context(16, "ch_ac", eps=0.05, tau=1e-5)
    st = A.empty_state(16)
    with pytest.raises(C.ChnsError):
        ctx.timestep_adjoint(A.fields_of(ctx, st), A.fields_of(ctx, st), A.fields_of(ctx, st),
                             A.fields_of(ctx, st))
    with pytest.raises(C.ChnsError):
        ctx.assemble_transposed(st["vel"])
    ctx.close()
    ctx = C.Context(16, "ternary", **BASE)
    f = A.fields_of(ctx, st)
    bad = ctx.fields(phi=[st["phi_p"]], mu=[st["mu_p"], st["mu_n"], st["mu_s"]], Phi_v=st["Phi"],
                     vel=st["vel"], p=st["p"])
    with pytest.raises(C.ChnsError):
        ctx.timestep_adjoint(f, f, bad, f)
    ctx.close()
