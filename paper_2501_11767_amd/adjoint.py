"""Differentiation form: ternary rollouts behind torch.autograd.

``rollout(ctx, theta, state0, steps, checkpoint, opts)`` advances the ternary
scheme ``steps`` steps from ``state0`` at parameters theta = (eps, mobility,
evaporation rate) and returns the final volume fractions (phi_p, phi_N).  Its
backward is the discrete adjoint of the scheme (``chns_timestep_adjoint``):
the forward pass keeps every ``checkpoint``-th state; the backward pass
recomputes one segment of states from its checkpoint at a time and runs the
adjoint steps through it in reverse, accumulating dL/dtheta and the adjoint of
the initial state.  ``mass_apply(ctx, x)`` is y = M x (symmetric), so the
M-weighted loss 1/2 sum_i (phi_i - t_i)^T M (phi_i - t_i) differentiates
through torch.

Every step, transposed solve and vector-Jacobian product runs in the HIP
library; this module only moves device pointers.
"""
from __future__ import annotations

import torch

from . import chns

FIELDS = ("phi_p", "phi_n", "mu_p", "mu_n", "mu_s", "Phi", "vel", "p")


def state_sizes(n: int):
    N = n * n
    return dict(phi_p=N, phi_n=N, mu_p=N, mu_n=N, mu_s=N, Phi=N, vel=8 * N, p=N)


def empty_state(n: int, device="cuda"):
    return {k: torch.zeros(v, dtype=torch.float64, device=device) for k, v in state_sizes(n).items()}


def fields_of(ctx: chns.Context, st):
    return ctx.fields(phi=[st["phi_p"], st["phi_n"]], mu=[st["mu_p"], st["mu_n"], st["mu_s"]],
                      Phi_v=st["Phi"], vel=st["vel"], p=st["p"])


def _set_theta(ctx: chns.Context, theta):
    t = [float(x) for x in theta.detach().cpu().tolist()]
    ctx.set_params(eps=t[0], mobility=t[1], evap_rate=t[2])


def _step(ctx, st, opts):
    nxt = {k: torch.empty_like(v) for k, v in st.items()}
    rc, info = ctx.timestep(fields_of(ctx, st), fields_of(ctx, nxt), 1, opts)
    if rc != chns.OK:
        raise chns.ChnsError(rc, f"forward step did not converge: {info}")
    return nxt


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta, ctx, steps, checkpoint, opts, adj_opts, *init):
        st = {k: v.detach() for k, v in zip(FIELDS, init)}
        _set_theta(ctx, theta)
        ckpts = {0: {k: v.clone() for k, v in st.items()}}
        for k in range(steps):
            st = _step(ctx, st, opts)
            if (k + 1) % checkpoint == 0 and k + 1 < steps:
                ckpts[k + 1] = {kk: v.clone() for kk, v in st.items()}
        fctx.ctx, fctx.steps, fctx.checkpoint = ctx, steps, checkpoint
        fctx.opts, fctx.adj_opts, fctx.ckpts = opts, adj_opts, ckpts
        fctx.save_for_backward(theta)
        fctx.infos = []
        return st["phi_p"].clone(), st["phi_n"].clone()

    @staticmethod
    def backward(fctx, g_php, g_phn):
        (theta,) = fctx.saved_tensors
        ctx, steps, K = fctx.ctx, fctx.steps, fctx.checkpoint
        _set_theta(ctx, theta)
        n = ctx.n
        lam = empty_state(n, device=g_php.device)
        lam["phi_p"].copy_(g_php)
        lam["phi_n"].copy_(g_phn)
        dtheta = torch.zeros(3, dtype=torch.float64)
        starts = sorted(fctx.ckpts)
        for s0 in reversed(starts):
            s1 = min(s0 + K, steps)
            seg = [fctx.ckpts[s0]]
            for _ in range(s0, s1):
                seg.append(_step(ctx, seg[-1], fctx.opts))
            for k in range(s1 - 1, s0 - 1, -1):
                rc, d, info = ctx.timestep_adjoint(fields_of(ctx, seg[k - s0]), fields_of(ctx, seg[k - s0 + 1]),
                                                   fields_of(ctx, lam), fields_of(ctx, lam), fctx.adj_opts)
                if rc != chns.OK:
                    raise chns.ChnsError(rc, f"adjoint step {k} did not converge: {info}")
                fctx.infos.append(info)
                dtheta += torch.from_numpy(d)
        grads_init = tuple(lam[k].clone() for k in FIELDS)
        return (dtheta.to(theta.device), None, None, None, None, None) + grads_init


def rollout(ctx: chns.Context, theta: torch.Tensor, state0: dict, steps: int, checkpoint: int = 10,
            opts=None, adj_opts=None):
    """(phi_p^N, phi_N^N) of a ternary run; differentiable in theta (and in
    the initial fields)."""
    if ctx.model != "ternary":
        raise ValueError("the differentiation form runs the ternary model")
    if steps < 1 or checkpoint < 1:
        raise ValueError("steps and checkpoint must be positive")
    o = opts or chns.default_opts(rtol=1e-10, precision=chns.MIXED, maxiter=1000)
    ao = adj_opts or o
    init = [state0[k] for k in FIELDS]
    return _Rollout.apply(theta, ctx, steps, checkpoint, o, ao, *init)


class _MassApply(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x, ctx):
        y = torch.empty_like(x)
        ctx.spmv(chns.OP_M, x.detach().contiguous(), y)
        fctx.ctx = ctx
        return y

    @staticmethod
    def backward(fctx, g):
        y = torch.empty_like(g)
        fctx.ctx.spmv(chns.OP_M, g.contiguous(), y)
        return y, None


def mass_apply(ctx: chns.Context, x: torch.Tensor) -> torch.Tensor:
    """y = M x with the P1 mass matrix (differentiable)."""
    return _MassApply.apply(x, ctx)


def loss(ctx: chns.Context, phis, targets) -> torch.Tensor:
    """1/2 sum_i (phi_i - t_i)^T M (phi_i - t_i)."""
    tot = None
    for ph, t in zip(phis, targets):
        d = ph - t
        term = 0.5 * torch.dot(d, mass_apply(ctx, d))
        tot = term if tot is None else tot + term
    return tot
