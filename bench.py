"""Benchmark of the coupled Cahn-Hilliard + Allen-Cahn step on one MI355X.

Workload (one "step" = one pass of the whole hot path): on the periodic
1024 x 1024 P1 mesh (1,048,576 nodes), assemble the step, build both
right-hand sides, solve the 2,097,152-unknown Cahn-Hilliard block with FGMRES
and the matching-Schur block preconditioner, and the 1,048,576-unknown
Allen-Cahn system with FGMRES and multigrid, to ||b - A x|| <= 1e-8 ||b||.
eps = 0.005, mobility 1, evaporation rate 0.1; initial phi = 0.4 +- 0.01
uniform noise, Phi_v = sin^2(pi y); tau = 1e-4 for the timed steps.

Prints one JSON line: DOF*iterations/s over the timed steps in the mixed
precision form (FP32 multigrid inside FP64 FGMRES), ms per step, the same for
plain FP64, a tau sweep {1e-5, 1e-4, 1e-3, 1e-2} with the error of both forms
against the oracle's exact Fourier-mode solve, the roofline of the dominant
kernel and the oracle's own FGMRES rate on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BATCH_RESTART = 60  # restart length of the batched workload and its sequential comparison
# multigrid of the batched workload and its sequential comparison: V(2,4) with
# the default cut (8 steps, rho <= 0.25); measured against V(2,2) (the library
# default), V(1,3), V(2,3), V(1,4), V(3,3), V(2,5), V(2,6), V(3,4), V(3,5),
# V(4,4), V(1,5), cut at rho <= 0.25/0.5/1/4 and 6-9 cut steps: V(2,4) is where
# more smoothing stops paying (batched eager step 73.1 -> 58.0 ms; the best,
# V(3,4), 56.6 ms)
BATCH_MG = dict(mg_pre=2, mg_post=4, mg_coarse=8, mg_rho_cut=0.25)
# multigrid of the 1024^2 workload: V(1,3), 8 Chebyshev steps on the cut level,
# hierarchies cut at the first level with rho <= 16 (measured fastest, summed
# over the tau sweep and two initial states, mixed and FP64, of V(1,2), V(1,3),
# V(2,2), V(2,3) with 7-9 cut steps; the library default is V(2,2), 8 steps,
# rho <= 0.25)
MG = dict(mg_pre=1, mg_post=3, mg_coarse=8, mg_rho_cut=16.0)
# the 256^2 ternary workload: the same multigrid with FGMRES(15) (restart 15
# measured fastest of 12/15/20 with this multigrid)
DRY_OPTS = dict(MG, restart=15)
# the cube's CH + AC step: FGMRES(13) (40^3 / 64^3 / 128^3 mixed steps 4.3 / 5.5 / 29.9 ms
# against 5.4 / 6.6 / 31.7 ms with 11)
CUBE_RESTART = 13
# the closed 10 x 10 square (box10): V(3,3) with FGMRES(20), measured fastest of V(1,3),
# V(2,2), V(2,4), V(3,3) with restarts 11, 13, 20 (3.45 ms at 32 CH iterations; V(1,3)
# with FGMRES(11): 4.7 ms at 62)
BOX_MG = dict(MG, mg_pre=3, mg_post=3)
BOX_RESTART = 20
# the paper's full two-dimensional run (quadbox, 65^2 vertices): FGMRES(30), the
# fastest of 15, 20, 30 with V(1,3) or V(2,2) (11.8 ms against 13.1 with 15)
QUADBOX_OPTS = dict(MG, restart=30)
# the closed-square workload: the 1024^2 multigrid with the cut threshold swept
# (its X operator has rho = 4 on the finest level, where the 1024^2 threshold
# would cut it to a four-step Chebyshev smoother)
BOX_RHO_CUTS = (16.0, 4.0, 1.0)
# HBM bytes per launch of a kernel from rocprofv3 counter runs of this
# benchmark (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a plain
# copy of known size); filled in from profiles/ once measured for the kernel
# as it stands, None otherwise.
TRAFFIC = {
    # profiles/chac1024_dcgs_update_hbm_counters.md: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0
    # per dispatch (the scales: the same counters on the 512 MiB negation probe)
    "k_dcgs_update": 152869730,
    # profiles/chac1024_tile_hbm_counters.md: the five finest-level tile passes
    # of a CH iteration (and the AC block's), averaged per launch like the ledger
    "k_vtile_pipe (finest-level tile passes; k_vtile in FP64)": 57340000,
}
METRIC = "solve DOF·iters/s + ms per coupled step, mixed vs FP64 at 1e-8; HBM GB/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--tau", type=float, default=1e-4)
    # FGMRES restart length of the 1024^2 workload: 11 measured fastest for the
    # mixed step at tau 1e-4 of 9-13 and 16 with its multigrid (the same 35 CH
    # iterations as 12 and 13)
    ap.add_argument("--restart", type=int, default=11)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ledger", action="store_true", help="no kernel events in the timed steps")
    ap.add_argument("--kernel-passes", action="store_true",
                    help="extra passes timing the other kernel classes (CH block, Gram-Schmidt)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="(default) the 512 MiB streaming probe: attainable bandwidth, counter calibration")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--dry-steps", type=int, default=5)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--box-steps", type=int, default=5)
    ap.add_argument("--quad-steps", type=int, default=5)
    ap.add_argument("--cube-steps", type=int, default=5)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-trajectory", action="store_true")
    ap.add_argument("--forms", default="mixed,fp64", help="timed forms of the 1024^2 step")
    return ap.parse_args()


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_steps(ctx, chns, fin, fout, k, opts):
    """k coupled steps, each from the seeded state `fin` into `fout` (the
    explicit potential term makes longer trajectories at these time steps
    diverge, so every timed step solves the same first-step systems);
    returns (wall ms list, infos list)."""
    import torch
    walls, infos = [], []
    for _ in range(k):
        t0 = time.perf_counter()
        rc, inf = ctx.timestep(fin, fout, 1, opts)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
        infos.append(inf)
        if rc < 0:
            raise RuntimeError(f"timestep failed: {rc}")
    return walls, infos


def dof_iters(infos, N):
    """Sum over solves of (unknowns x iterations) and of solve ms."""
    di, ms = 0.0, 0.0
    for inf in infos:
        ch, ac = inf[0], inf[1]
        di += 2 * N * ch["iters"] + N * ac["iters"]
        ms += ch["ms"] + ac["ms"]
    return di, ms


def ledger_figures(led, k):
    launches, nbytes, ms = led
    gbs = nbytes / (ms * 1e-3) / 1e9
    return dict(launches=launches, ms_total=ms, ms_per_step=ms / k, us_per_launch=ms * 1e3 / launches,
                bytes_per_launch=nbytes / launches, gbs=gbs, frac=gbs / HBM_PEAK_GBS)


def kernel_ledger(ctx, chns, fin, fout, k, opts, all_classes=False):
    """Per kernel class: the same k timed steps again with the library's
    ledger on, which launches every kernel of the class with a pair of HIP
    events timestamped by the dispatch itself, on the stream it runs on (the
    library launches on torch's current stream), and records its algorithmic
    bytes.  Always the roofline class (the Gram-Schmidt update pass), the CH
    block operator and the finest-level multigrid passes; with all_classes
    also the dot pass and the launch-per-step Chebyshev sweeps.  The events
    cost the step time, so these passes are separate from the value pass; on
    short kernels (~3-10 us) they also lengthen the kernels themselves, so
    those figures are indicative only.  Returns {kernel name: figures}."""
    out = {}
    classes = [chns.KERNEL_DCGS_UPDATE, chns.KERNEL_CH_BLOCK, chns.KERNEL_MG_FINE]
    if all_classes:
        classes += [chns.KERNEL_DCGS_DOTS, chns.KERNEL_CHEB32]
    for kid in classes:
        ctx.ledger_start(kid)
        run_steps(ctx, chns, fin, fout, k, opts)
        led = ctx.ledger_read()
        ctx.ledger_start(-1)
        if led[0]:
            out[chns.KERNEL_NAMES[kid]] = ledger_figures(led, k)
    return out


def copy_probe(mib=512, reps=9):
    """One plain streaming kernel of known traffic (b = -a over 512 MiB FP32,
    torch's elementwise negation): its event-timed median gives the streaming
    bandwidth this GPU attains in practice, and in a profiled run its
    FETCH_SIZE / WRITE_SIZE per dispatch scale the HBM counters."""
    import torch
    a = torch.ones(mib * 2 ** 18, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.neg(a, out=b)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.neg(a, out=b)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = sorted(ts)[reps // 2]
    nbytes = 2 * a.numel() * 4
    out = dict(kernel="neg (elementwise)", bytes_read=a.numel() * 4, bytes_written=b.numel() * 4,
               dispatches=reps + 1, us=ms * 1e3, gbs=nbytes / (ms * 1e6), frac=nbytes / (ms * 1e6) / HBM_PEAK_GBS)
    del a, b
    torch.cuda.empty_cache()
    return out


def cpu_baseline(cfg, n, tau, budget_s=20.0):
    """The oracle's flexible GMRES with its multigrid block preconditioner on
    the same CH system, a bounded number of Arnoldi steps, single thread."""
    from threadpoolctl import threadpool_limits

    from oracle import fem, krylov, precond as PC, systems
    from oracle.systems import Params
    from paper_2501_11767_amd import inputs
    with threadpool_limits(1):
        t0 = time.perf_counter()
        m = fem.Mesh(n)
        M, K = fem.p1_mass(m), fem.p1_stiffness(m)
        prm = Params(eps=cfg["eps"], tau=tau, mobility=cfg["mobility"], evap_rate=cfg["evap_rate"])
        f = inputs.initial_state(n, "ch_ac", cfg["mean"], cfg["seed"])
        from oracle import potential as pot
        A = systems.ch_matrix(M, K, None, prm)
        b = systems.ch_rhs(M, f["phi"][0], pot.dfdphi_bin(f["phi"][0], f["Phi_v"]), prm)
        P = PC.CHPreconditioner(M, K, None, prm, n, inner="mg", rho_cut=MG["mg_rho_cut"], pre=MG["mg_pre"],
                                post=MG["mg_post"], coarse=MG["mg_coarse"])
        setup = time.perf_counter() - t0
        # one Arnoldi step to size the sample, then as many as fit the budget
        t1 = time.perf_counter()
        krylov.fgmres(A, b, prec=P.apply, fixed_iters=1)
        one = time.perf_counter() - t1
        k = int(max(1, min(30, (budget_s - setup) / max(one, 1e-3))))
        t2 = time.perf_counter()
        krylov.fgmres(A, b, prec=P.apply, fixed_iters=k)
        dt = time.perf_counter() - t2
    N2 = 2 * n * n
    return dict(value=N2 * k / dt, unit="DOF·iters/s", cores=1, kind="oracle",
                sample=f"oracle FGMRES + V({MG['mg_pre']},{MG['mg_post']}) block preconditioner, CH system of the "
                       f"{n}x{n} mesh ({N2} unknowns), {k} Arnoldi steps in {dt:.1f} s "
                       f"after {setup:.1f} s of set-up, FP64, 1 thread")


def trajectory_section(chns, ctx, st0, p, args, tau=1e-5, steps=10):
    """A real trajectory of the 1024^2 workload: `steps` consecutive steps from
    the seeded state at tau = 1e-5 (the explicit potential term keeps this tau
    stable; at the benchmark's tau = 1e-4 the trajectory blows up within ~10
    steps), each step solving the previous step's output, so the solver meets
    a new system every step and its rate predictor the history of the last."""
    import torch
    N = args.n * args.n
    out = {}
    ctx.set_params(**dict(p, tau=tau))
    for name, prec in (("mixed", chns.MIXED), ("fp64", chns.F64)):
        phi, Phi = dev(st0["phi"][0]), dev(st0["Phi_v"])
        mu = torch.zeros(N, dtype=torch.float64, device="cuda")
        f = ctx.fields(phi=[phi], mu=[mu], Phi_v=Phi)
        opts = chns.default_opts(rtol=1e-8, precision=prec, restart=args.restart, **MG)
        d0 = ctx.diagnostics(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, infos = ctx.timestep(f, f, steps, opts)
        torch.cuda.synchronize()
        total = (time.perf_counter() - t0) * 1e3
        d1 = ctx.diagnostics(f)
        out[name] = dict(ms_per_step=total / steps, ch_iters=[i["iters"] for i in infos[0::2]],
                         ac_iters=[i["iters"] for i in infos[1::2]],
                         converged=all(i["converged"] for i in infos),
                         mass_phi_rel_change=(d1[0] - d0[0]) / d0[0], energy=[d0[4], d1[4]])
    ctx.set_params(**p)
    return dict(workload=f"chac{args.n} trajectory: {steps} consecutive steps in place from the seeded state at "
                         f"tau {tau}, rtol 1e-8, the benchmark's solver options", **out)


def dry_section(chns, steps):
    """The full coupled drying step (two CH phases, AC, Taylor-Hood Oseen) on the
    periodic 256 x 256 mesh in plain FP64: ms per coupled step and FGMRES
    iterations per solve, each step from the seeded state (at tau = 5e-4 the
    explicit potential makes the trajectory diverge within 20 steps).  mu^0 = 0
    (only an initial guess and the alpha-scaled convecting term; alpha = 1e-8)."""
    import torch
    from paper_2501_11767_amd import inputs
    cfg = inputs.CONFIGS["dry256"]
    n = cfg["n"]
    N = n * n
    ctx = chns.Context(n, "ternary", eps=cfg["eps"], tau=cfg["tau"], mobility=cfg["mobility"],
                       evap_rate=cfg["evap_rate"], viscosity=cfg["viscosity"], alpha=1e-8, rho=1.0)
    st = inputs.initial_state(n, "ternary", cfg["mean"], cfg["seed"])
    z = lambda: torch.zeros(N, dtype=torch.float64, device="cuda")
    fld = dict(phi=[dev(st["phi"][0]), dev(st["phi"][1])], mu=[z(), z(), z()],
               Phi_v=dev(st["Phi_v"]), vel=dev(st["vel"].ravel()), p=dev(st["p"]))
    f = ctx.fields(**fld)
    e = lambda k: torch.empty(k, dtype=torch.float64, device="cuda")
    fo = ctx.fields(phi=[e(N), e(N)], mu=[e(N), e(N), e(N)], Phi_v=e(N), vel=e(8 * N), p=e(N))
    opts = chns.default_opts(rtol=1e-8, precision=chns.F64, maxiter=1000, **DRY_OPTS)
    ctx.timestep(f, fo, 1, opts)  # warm-up step
    torch.cuda.synchronize()
    walls, its = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        rc, inf = ctx.timestep(f, fo, 1, opts)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
        its.append([i["iters"] for i in inf])
    ctx.close()
    return dict(baseline_config="full coupled drying step, 20 time steps on 256x256 P1/Taylor-Hood, FP64, "
                                "eps 0.01, tau 5e-4",
                as_run=f"{steps} timed steps after one warm-up, each re-solving the seeded first step: at tau 5e-4 "
                       "the explicit potential term makes the 20-step trajectory blow up (the 1024^2 parameters "
                       "do within 8 steps at tau 1e-4 on the CPU, tests/test_oracle_step.py::"
                       "test_explicit_potential_limits_the_time_step)",
                workload=f"dry256: ternary CH + AC + Taylor-Hood Oseen step, periodic {n}x{n} "
                         f"({2 * 2 * N} CH + {N} AC + {9 * N} NS unknowns), FP64, FGMRES({DRY_OPTS['restart']}) "
                         f"rtol 1e-8, V({MG['mg_pre']},{MG['mg_post']}) multigrid cut at rho <= {MG['mg_rho_cut']}",
                ms_per_step=float(np.mean(walls)), ms_per_step_median=float(np.median(walls)),
                iters_ch_p_ch_n_ac_ns=its, steps=steps)


def quad_section(chns, steps):
    """The paper's full system on the periodic 256 x 256 mesh (quad256): three
    CH phases with their own beta, AC, Taylor-Hood Oseen, air closure, in
    plain FP64 with the drying workload's solver options: ms per coupled step
    and FGMRES iterations, each step from the seeded state (mu^0 = 0)."""
    import torch
    from paper_2501_11767_amd import inputs
    cfg = inputs.CONFIGS["quad256"]
    n = cfg["n"]
    N = n * n
    ctx = chns.Context(n, "quaternary", eps=cfg["eps"], tau=cfg["tau"], mobility=cfg["mobility"],
                       evap_rate=cfg["evap_rate"], viscosity=cfg["viscosity"], alpha=cfg["alpha"], rho=1.0,
                       beta_phase=cfg["betas"])
    st = inputs.initial_state(n, "quaternary", cfg["mean"], cfg["seed"])
    z = lambda: torch.zeros(N, dtype=torch.float64, device="cuda")
    f = ctx.fields(phi=[dev(st["phi"][i]) for i in range(3)], mu=[z(), z(), z(), z()], Phi_v=dev(st["Phi_v"]),
                   vel=dev(st["vel"].ravel()), p=dev(st["p"]))
    e = lambda k: torch.empty(k, dtype=torch.float64, device="cuda")
    fo = ctx.fields(phi=[e(N), e(N), e(N)], mu=[e(N), e(N), e(N), e(N)], Phi_v=e(N), vel=e(8 * N), p=e(N))
    opts = chns.default_opts(rtol=1e-8, precision=chns.F64, maxiter=1000, **DRY_OPTS)
    ctx.timestep(f, fo, 1, opts)
    torch.cuda.synchronize()
    walls, its = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        rc, inf = ctx.timestep(f, fo, 1, opts)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
        its.append([i["iters"] for i in inf])
    ctx.close()
    b = cfg["betas"]
    return dict(workload=f"quad256: quaternary CH (polymer, NFA, solvent; air eliminated) + AC + Taylor-Hood "
                         f"Oseen step, periodic {n}x{n} ({3 * 2 * N} CH + {N} AC + {9 * N} NS unknowns), FP64, "
                         f"beta_p,N,s,a {b}, beta_v {cfg['eps'] ** 2:.0e}, tau {cfg['tau']}, FGMRES("
                         f"{DRY_OPTS['restart']}) rtol 1e-8, V({MG['mg_pre']},{MG['mg_post']}) multigrid",
                ms_per_step=float(np.mean(walls)), ms_per_step_median=float(np.median(walls)),
                iters_ch_p_ch_n_ch_s_ac_ns=its[-1], steps=steps)


def quadbox_section(chns, steps):
    """The paper's full two-dimensional run (quadbox): the quaternary step on
    the closed 10 x 10 square with no-flux and no-slip walls, FP64 with the
    drying workload's solver options: ms per coupled step and FGMRES
    iterations, each step from the seeded state (mu^0 = 0)."""
    import torch
    from paper_2501_11767_amd import inputs
    cfg = inputs.CONFIGS["quadbox"]
    n, L = cfg["n"], cfg["length"]
    ctx = chns.Context(n, "quaternary", boundary="noflux", length=L, eps=cfg["eps"], tau=cfg["tau"],
                       mobility=cfg["mobility"], evap_rate=cfg["evap_rate"], viscosity=cfg["viscosity"],
                       alpha=cfg["alpha"], rho=1.0, beta_phase=cfg["betas"])
    N = ctx.N
    st = inputs.box_state(n, L, "quaternary", cfg["mean"], cfg["seed"])
    z = lambda: torch.zeros(N, dtype=torch.float64, device="cuda")
    f = ctx.fields(phi=[dev(st["phi"][i]) for i in range(3)], mu=[z(), z(), z(), z()], Phi_v=dev(st["Phi_v"]),
                   vel=dev(st["vel"].ravel()), p=dev(st["p"]))
    e = lambda k: torch.empty(k, dtype=torch.float64, device="cuda")
    fo = ctx.fields(phi=[e(N), e(N), e(N)], mu=[e(N), e(N), e(N), e(N)], Phi_v=e(N), vel=e(8 * N), p=e(N))
    opts = chns.default_opts(rtol=1e-8, precision=chns.F64, maxiter=1000, **QUADBOX_OPTS)
    ctx.timestep(f, fo, 1, opts)
    torch.cuda.synchronize()
    walls, its = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        rc, inf = ctx.timestep(f, fo, 1, opts)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
        its.append([i["iters"] for i in inf])
    ctx.close()
    return dict(workload=f"quadbox: quaternary CH + AC + Taylor-Hood Oseen step on the closed square [0, {L}]^2 "
                         f"(no-flux walls, no-slip velocity), {n} cells per side ({N} vertices), betas "
                         f"{cfg['betas']}, beta_v = delta_v = {cfg['eps'] ** 2:g}, tau {cfg['tau']}, FP64, FGMRES("
                         f"{QUADBOX_OPTS['restart']}) rtol 1e-8",
                ms_per_step=float(np.mean(walls)), ms_per_step_median=float(np.median(walls)),
                iters_ch_p_ch_n_ch_s_ac_ns=its[-1], steps=steps)


def box_section(chns, steps, restart):
    """The paper's closed domain: the CH + AC step on the 10 x 10 square with
    no-flux walls (128 cells per side, 129^2 vertices, film under air),
    mixed precision with the 1024^2 workload's solver options: ms per step
    and FGMRES iterations, each step from the seeded state (mu^0 = 0: in the
    binary step it is only the Krylov initial guess)."""
    import torch
    from paper_2501_11767_amd import inputs
    cfg = inputs.CONFIGS["box10"]
    n, L = cfg["n"], cfg["length"]
    p = {k: cfg[k] for k in ("eps", "tau", "mobility", "evap_rate")}
    ctx = chns.Context(n, "ch_ac", boundary="noflux", length=L, **p)
    st = inputs.box_state(n, L, "ch_ac", cfg["mean"], cfg["seed"])
    N = ctx.N
    f = ctx.fields(phi=[dev(st["phi"][0])], mu=[torch.zeros(N, dtype=torch.float64, device="cuda")],
                   Phi_v=dev(st["Phi_v"]))
    e = lambda: torch.empty(N, dtype=torch.float64, device="cuda")
    fo = ctx.fields(phi=[e()], mu=[e()], Phi_v=e())
    by_cut = {}
    for cut in BOX_RHO_CUTS:
        opts = chns.default_opts(rtol=1e-8, precision=chns.MIXED, restart=restart, **dict(BOX_MG, mg_rho_cut=cut))
        ctx.timestep(f, fo, 1, opts)
        torch.cuda.synchronize()
        walls, its = [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            rc, inf = ctx.timestep(f, fo, 1, opts)
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t0) * 1e3)
            its.append([i["iters"] for i in inf])
        by_cut[cut] = dict(ms_per_step=float(np.mean(walls)), ms_per_step_median=float(np.median(walls)),
                           iters_ch_ac=its[-1])
    ctx.close()
    best = min(by_cut, key=lambda k: by_cut[k]["ms_per_step"])
    return dict(workload=f"box10: CH + AC step on the closed square [0, {L}]^2 with no-flux walls, {n} cells "
                         f"per side ({N} vertices, {3 * N} unknowns), film at {cfg['mean']} +- 0.01 under air, "
                         f"eps^2 {cfg['eps'] ** 2:.3g}, tau {cfg['tau']}, mixed precision, FGMRES({restart}) "
                         f"rtol 1e-8, V({BOX_MG['mg_pre']},{BOX_MG['mg_post']}) multigrid; per hierarchy cut threshold",
                rho_cut=best, **by_cut[best], by_rho_cut={str(k): v for k, v in by_cut.items()}, steps=steps)


def cube_section(chns, steps, restart):
    """The paper's three-dimensional grid: the CH + AC step on the periodic
    cube (Kuhn tetrahedra, 15-entry P1 rows) at 40 cells per side and the
    larger sizes, mixed precision with the 1024^2 workload's solver options:
    ms per step and FGMRES iterations per hierarchy cut threshold, each step
    from the seeded state (mu^0 = 0, the Krylov initial guess)."""
    import torch
    from paper_2501_11767_amd import inputs
    cfg = inputs.CONFIGS["cube40"]
    bcfg = inputs.CONFIGS["cubebox40"]
    p = {k: cfg[k] for k in ("eps", "tau", "mobility", "evap_rate")}
    bp = {k: bcfg[k] for k in ("eps", "tau", "mobility", "evap_rate")}
    out = {}
    cases = [(str(n), n, False) for n in cfg["sizes"]] + [("closed40", bcfg["n"], True)]
    for name, n, closed in cases:
        t0 = time.perf_counter()
        if closed:
            ctx = chns.Context(n, "ch_ac", dim=3, boundary="noflux", length=bcfg["length"], **bp)
            st = inputs.cube_box_state(n, bcfg["length"], "ch_ac", bcfg["mean"], bcfg["seed"])
        else:
            ctx = chns.Context(n, "ch_ac", dim=3, **p)
            st = inputs.cube_state(n, "ch_ac", cfg["mean"], cfg["seed"])
        log(f"cube {name}: create {time.perf_counter() - t0:.1f} s")
        N = ctx.N
        f = ctx.fields(phi=[dev(st["phi"][0])], mu=[torch.zeros(N, dtype=torch.float64, device="cuda")],
                       Phi_v=dev(st["Phi_v"]))
        e = lambda: torch.empty(N, dtype=torch.float64, device="cuda")
        fo = ctx.fields(phi=[e()], mu=[e()], Phi_v=e())
        by_cut = {}
        for cut in BOX_RHO_CUTS:
            opts = chns.default_opts(rtol=1e-8, precision=chns.MIXED, restart=restart, **dict(MG, mg_rho_cut=cut))
            ctx.timestep(f, fo, 1, opts)
            torch.cuda.synchronize()
            walls, its = [], []
            for _ in range(steps):
                t0 = time.perf_counter()
                rc, inf = ctx.timestep(f, fo, 1, opts)
                torch.cuda.synchronize()
                walls.append((time.perf_counter() - t0) * 1e3)
                its.append([i["iters"] for i in inf])
            by_cut[cut] = dict(ms_per_step=float(np.mean(walls)), ms_per_step_median=float(np.median(walls)),
                               iters_ch_ac=its[-1])
        ctx.close()
        best = min(by_cut, key=lambda k: by_cut[k]["ms_per_step"])
        b = by_cut[best]
        out[name] = dict(nodes=N, unknowns=3 * N, rho_cut=best, **b,
                           dof_iters_per_s=3 * N * sum(b["iters_ch_ac"]) / (b["ms_per_step"] * 1e-3),
                           by_rho_cut={str(k): v for k, v in by_cut.items()})
    return dict(workload=f"cube40: CH + AC step on the periodic unit cube, Kuhn tetrahedra, "
                         f"{cfg['sizes']} cells per side (40 is the paper's grid), phase at {cfg['mean']} +- 0.01, "
                         f"vapour layer sin^2(pi z), eps {cfg['eps']}, tau {cfg['tau']}, mixed precision, "
                         f"FGMRES({restart}) rtol 1e-8, V({MG['mg_pre']},{MG['mg_post']}) multigrid; per size the "
                         f"best hierarchy cut threshold; 'closed40': the paper's closed [0, {bcfg['length']}]^3 cube "
                         f"with no-flux walls on its 40^3 grid ((41)^3 vertices), film z <= 5 at {bcfg['mean']} +- 0.01 "
                         f"under air, eps^2 {bcfg['eps'] ** 2:.3g}, tau {bcfg['tau']}", sizes=out, steps=steps)


def batch_section(chns, steps):
    """64 independent CH + AC instances (sizes drawn from {64, 128, 256, 512}^2,
    parameters log-uniform) advanced together: FP32 multigrid inside FP64
    FGMRES, autotuned launch shapes, `steps` steps captured in one hipGraph
    (each step solves the seeded first-step systems).  Compared with the
    plain FP64 solve of the same 64 steps one instance at a time."""
    import torch
    from paper_2501_11767_amd import inputs
    inst = inputs.batch_instances()
    sizes = [d["n"] for d in inst]
    prm = [dict(eps=d["eps"], tau=d["tau"], mobility=d["mobility"], evap_rate=d["evap_rate"])
           for d in inst]
    phi0, Phi0 = [], []
    for d in inst:
        st = inputs.initial_state(d["n"], "ch_ac", 0.4, d["seed"])
        phi0.append(st["phi"][0])
        Phi0.append(st["Phi_v"])
    phi0, Phi0 = np.concatenate(phi0), np.concatenate(Phi0)
    Ntot = len(phi0)
    log(f"batch64: create ({Ntot} nodes)")
    t0 = time.perf_counter()
    batch = chns.Batch(sizes, prm)
    setup = time.perf_counter() - t0
    s = torch.cuda.Stream()
    zin = [dev(phi0), torch.zeros(Ntot, dtype=torch.float64, device="cuda"), dev(Phi0)]
    out = [torch.empty(Ntot, dtype=torch.float64, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    log("batch64: tune")
    batch.tune(None, stream=s)
    opts = chns.default_opts(rtol=1e-8, precision=chns.MIXED, restart=BATCH_RESTART, maxiter=120, **BATCH_MG)
    log("batch64: eager steps")
    rc_e, info_e = batch.timestep(*zin, nsteps=steps, opts=opts, use_graph=False, stream=s, out=out,
                                  each_from_input=True)
    eager_ms = info_e["ms"] / steps
    # graph budgets from the eager step, one step captured and replayed
    batch.calibrate_graph(info_e)
    log(f"batch64: graph capture ({steps} steps in one graph) and a first replay")
    batch.timestep(*zin, nsteps=steps, opts=opts, use_graph=True, stream=s, out=out, each_from_input=True)
    log("batch64: graph steps")
    rc, info = batch.timestep(*zin, nsteps=steps, opts=opts, use_graph=True, stream=s, out=out,
                              each_from_input=True)
    graph_ms = info["ms"] / steps
    upd_threads, dots_group = batch.tuned()
    # the same steps with the work-list form of the tiled multigrid passes (a
    # grid of one workgroup per CU taking tiles from atomic counters)
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    batch.set_worklist(ncu)
    log("batch64: work-list form, eager and graph steps")
    _, info_we = batch.timestep(*zin, nsteps=steps, opts=opts, use_graph=False, stream=s, out=out,
                                each_from_input=True)
    batch.timestep(*zin, nsteps=steps, opts=opts, use_graph=True, stream=s, out=out, each_from_input=True)
    _, info_wg = batch.timestep(*zin, nsteps=steps, opts=opts, use_graph=True, stream=s, out=out,
                                each_from_input=True)
    worklist = dict(grid=ncu, eager_ms_per_step=info_we["ms"] / steps, graph_ms_per_step=info_wg["ms"] / steps)
    batch.set_worklist(0)
    log("batch64: fp64 eager step")
    o64 = chns.default_opts(rtol=1e-8, precision=chns.F64, restart=BATCH_RESTART, maxiter=120, **BATCH_MG)
    rc_f, info_f = batch.timestep(*zin, nsteps=1, opts=o64, use_graph=False, stream=s, out=out)
    batch.close()
    di = float(sum(2 * n * n * a + n * n * b for n, a, b in zip(sizes, info["iters_ch"], info["iters_ac"])))
    # one instance at a time, plain FP64, one context per size
    ctxs, seq_ms, seq_its = {}, 0.0, 0
    off = np.concatenate([[0], np.cumsum([n * n for n in sizes])])
    opts_seq = chns.default_opts(rtol=1e-8, precision=chns.F64, restart=BATCH_RESTART, maxiter=600, **BATCH_MG)
    log("batch64: sequential fp64 solves")
    for i, (n, p) in enumerate(zip(sizes, prm)):
        if n not in ctxs:
            ctxs[n] = chns.Context(n, "ch_ac", **p)
        c = ctxs[n]
        c.set_params(**p)
        sl = slice(int(off[i]), int(off[i + 1]))
        fi = c.fields(phi=[zin[0][sl].contiguous()], mu=[zin[1][sl].contiguous()], Phi_v=zin[2][sl].contiguous())
        fo = c.fields(phi=[out[0][sl].contiguous()], mu=[out[1][sl].contiguous()], Phi_v=out[2][sl].contiguous())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, inf = c.timestep(fi, fo, 1, opts_seq)
        torch.cuda.synchronize()
        seq_ms += (time.perf_counter() - t1) * 1e3
        seq_its += inf[0]["iters"]
    for c in ctxs.values():
        c.close()
    return dict(baseline_config="64 independent coupled-step instances, sizes from {64..512}^2, log-uniform "
                                "parameters, FP32 preconditioner in FP64 FGMRES, one persistent launch, "
                                "hipGraph-captured over 10 steps, tile and slice parameters from the autotuner",
                as_run=f"{steps} steps captured in one hipGraph and replayed; every step solves the seeded "
                       "first-step systems (the explicit potential term limits the stable tau, see the 1024^2 "
                       "workload); one launch per stage over all instances (the persistent variant is measured "
                       "separately); autotuned smoothing shapes per level and Gram-Schmidt shapes",
                tuned_update_threads=upd_threads, tuned_dots_group=dots_group, worklist_form=worklist,
                workload=f"batch64: 64 CH + AC instances, sizes {sorted(set(sizes))} "
                         f"({Ntot} nodes, {3 * Ntot} unknowns), log-uniform eps, tau, mobility, "
                         f"evaporation rate; FP32 V({BATCH_MG['mg_pre']},{BATCH_MG['mg_post']}) multigrid in FP64 "
                         f"FGMRES({BATCH_RESTART}), rtol 1e-8",
                graph_ms_per_step=graph_ms, eager_ms_per_step=eager_ms,
                graph_budget_ch_ac=[int(x.max()) for x in (info_e["iters_ch"], info_e["iters_ac"])],
                sequential_fp64_ms_per_step=seq_ms, speedup_vs_sequential_fp64=seq_ms / graph_ms,
                dof_iters_per_s=di / (graph_ms * 1e-3),
                converged=int(info["conv_ch"].sum() + info["conv_ac"].sum()), solves=2 * len(sizes),
                batch_fp64_converged=int(info_f["conv_ch"].sum() + info_f["conv_ac"].sum()),
                iters_ch_max=int(info["iters_ch"].max()), iters_ch_mean=float(info["iters_ch"].mean()),
                sequential_fp64_iters_ch_mean=seq_its / len(sizes), setup_s=setup, graph_steps=steps)


def adjoint_state0(n, cfg):
    """Seeded initial state of the differentiation workload (mu^0 = p^0 = 0)."""
    import torch
    from paper_2501_11767_amd import inputs
    f = inputs.initial_state(n, "ternary", cfg["mean"], cfg["seed"])
    z = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda")
    N = n * n
    return dict(phi_p=dev(f["phi"][0]), phi_n=dev(f["phi"][1]), mu_p=z(N), mu_n=z(N), mu_s=z(N),
                Phi=dev(f["Phi_v"]), vel=dev(np.asarray(f["vel"]).ravel()), p=z(N))


def adjoint_section(chns):
    """Differentiation form on the 128 x 128 ternary workload: 50 steps,
    checkpoint every 10, loss = M-weighted L2 mismatch of the final volume
    fractions to the run at theta_ref; gradient at theta0 by the adjoint
    (FP64 FGMRES, FP32 multigrid, rtol 1e-10) against central differences
    with absolute step 1e-6 (FP64 solves at rtol 1e-13)."""
    import torch
    from paper_2501_11767_amd import adjoint as A, inputs
    cfg = inputs.CONFIGS["adjoint128"]
    n, steps, K = cfg["n"], cfg["steps"], cfg["checkpoint"]
    ref = (cfg["eps"], cfg["mobility"], cfg["evap_rate"])
    th0 = tuple(cfg["theta0"])
    ctx = chns.Context(n, "ternary", eps=ref[0], tau=cfg["tau"], mobility=ref[1], evap_rate=ref[2],
                       viscosity=cfg["viscosity"], alpha=cfg["alpha"], rho=1.0)
    st0 = adjoint_state0(n, cfg)
    tight = chns.default_opts(rtol=1e-13, precision=chns.F64, maxiter=3000)
    mixed = chns.default_opts(rtol=1e-10, precision=chns.MIXED, maxiter=2000)

    def final(theta, opts):
        with torch.no_grad():
            th = torch.tensor(theta, dtype=torch.float64)
            return A.rollout(ctx, th, st0, steps, checkpoint=K, opts=opts)

    log("adjoint128: target run at theta_ref")
    target = [t.clone() for t in final(ref, tight)]

    def loss_at(theta, opts):
        php, phn = final(theta, opts)
        return float(A.loss(ctx, (php, phn), target))

    res = {}
    for name, opts in (("mixed", mixed), ("fp64", tight)):
        log(f"adjoint128: rollout + adjoint at theta0 ({name})")
        theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        php, phn = A.rollout(ctx, theta, st0, steps, checkpoint=K, opts=opts)
        L = A.loss(ctx, (php, phn), target)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res[name] = dict(loss=float(L.detach()), grad=theta.grad.tolist(), forward_ms=(t1 - t0) * 1e3,
                         backward_ms=(t2 - t1) * 1e3)
    log("adjoint128: central differences")

    def central(opts, h=1e-6):
        out = []
        for j in range(3):
            tp, tm = list(th0), list(th0)
            tp[j] += h
            tm[j] -= h
            out.append((loss_at(tp, opts) - loss_at(tm, opts)) / (2 * h))
        return out
    fd = central(tight)
    # the quotient's noise floor: the loss carries the forward solves' error
    # (rtol 1e-13), which the quotient divides by 2h; estimated by the change of
    # the loss and of the quotient when the solves are tightened to 1e-14
    tighter = chns.default_opts(rtol=1e-14, precision=chns.F64, maxiter=6000)
    try:
        fd_t = central(tighter)
        dL = abs(loss_at(th0, tight) - loss_at(th0, tighter))
    except chns.ChnsError as e:  # 1e-14 below this system's residual floor
        log(f"adjoint128: solves at rtol 1e-14 did not converge ({e}); no noise-floor estimate")
        fd_t, dL = None, None
    # fourth-order differences with relative steps 1e-3 (truncation O(h^4)):
    # the evaporation-rate derivative is ~1e-10, so with h = 1e-6 the
    # difference quotient is limited by the rounding of L itself
    fd4 = []
    for j in range(3):
        h = 1e-3 * th0[j]
        at = lambda k: loss_at([th0[i] + (k * h if i == j else 0.0) for i in range(3)], tight)
        fd4.append((-at(2) + 8 * at(1) - 8 * at(-1) + at(-2)) / (12 * h))
    L_ref = loss_at(ref, tight)
    floor = None if dL is None else [2 * dL / (2 * 1e-6) / abs(b) for b in fd]  # relative, per parameter
    for name in ("mixed", "fp64"):
        g = res[name]["grad"]
        res[name]["rel_err_vs_fd"] = [abs(a - b) / abs(b) for a, b in zip(g, fd)]
        res[name]["rel_err_vs_fd_rtol1e-14"] = None if fd_t is None else [abs(a - b) / abs(b)
                                                                          for a, b in zip(g, fd_t)]
        res[name]["rel_err_vs_fd4"] = [abs(a - b) / abs(b) for a, b in zip(g, fd4)]
    ctx.close()
    return dict(workload=f"adjoint128: ternary CH + AC + Oseen, periodic {n}x{n}, {steps} steps at "
                         f"tau {cfg['tau']} (the stated 1e-3 diverges with the explicit potential), "
                         f"checkpoint every {K}; loss = 1/2 sum_i |phi_i^N - target_i|_M^2, target from "
                         f"theta_ref = {ref}; gradient at theta0 = {th0}",
                baseline_config="ternary CH-AC-NS, 128x128, 50 steps at tau 1e-3, checkpoint every 10, "
                                "gradients vs central differences (h 1e-6) and the CPU FP64 gradient",
                as_run="50 steps at tau 3e-6: at tau 1e-3 the explicit potential term makes the scheme blow up "
                       "within 3 steps (CPU, direct solves: tests/test_oracle_step.py::"
                       "test_explicit_potential_limits_the_time_step)",
                theta0=list(th0), fd_grad=fd, fd_grad_rtol1e_14=fd_t, fd_step=1e-6,
                loss_change_rtol_1e13_to_1e14=dL, fd_noise_floor_rel=floor, fd4_grad=fd4, fd4_rel_step=1e-3,
                loss_at_ref=L_ref, **res)


def cpu_adjoint_reference(chns, n=16, steps=10):
    """CPU leg: the oracle's FP64 reverse-sweep gradient on a bounded sample
    of the differentiation workload (same parameters, n x n, `steps` steps)
    next to the GPU adjoint on the same sample."""
    import torch
    from oracle import adjoint as AD, step as S
    from oracle.systems import Params
    from paper_2501_11767_amd import adjoint as A, inputs
    cfg = inputs.CONFIGS["adjoint128"]
    ref = dict(eps=cfg["eps"], tau=cfg["tau"], mobility=cfg["mobility"], evap_rate=cfg["evap_rate"],
               viscosity=cfg["viscosity"], alpha=cfg["alpha"])
    th0 = dict(ref, eps=cfg["theta0"][0], mobility=cfg["theta0"][1], evap_rate=cfg["theta0"][2])
    f = inputs.initial_state(n, "ternary", cfg["mean"], cfg["seed"])
    N = n * n
    st0 = dict(phi=[f["phi"][0], f["phi"][1]], mu=[np.zeros(N), np.zeros(N)], mu_s=np.zeros(N),
               Phi_v=f["Phi_v"], vel=np.asarray(f["vel"]).reshape(2, 4 * N), p=np.zeros(N))
    ops = S.Operators(n, need_p2=True)
    t0 = time.perf_counter()
    target = AD.rollout(ops, Params(**ref), st0, steps)[-1]["phi"]
    L, g = AD.gradient(ops, Params(**th0), st0, target, steps)
    cpu_s = time.perf_counter() - t0
    ctx = chns.Context(n, "ternary", **dict(th0, rho=1.0))
    theta = torch.tensor([th0["eps"], th0["mobility"], th0["evap_rate"]], dtype=torch.float64,
                         requires_grad=True)
    s0 = dict(phi_p=dev(st0["phi"][0]), phi_n=dev(st0["phi"][1]), mu_p=dev(st0["mu"][0]),
              mu_n=dev(st0["mu"][1]), mu_s=dev(st0["mu_s"]), Phi=dev(st0["Phi_v"]),
              vel=dev(st0["vel"].ravel()), p=dev(st0["p"]))
    opts = chns.default_opts(rtol=1e-13, precision=chns.F64, maxiter=3000)
    php, phn = A.rollout(ctx, theta, s0, steps, checkpoint=cfg["checkpoint"], opts=opts)
    Lg = A.loss(ctx, (php, phn), (dev(target[0]), dev(target[1])))
    Lg.backward()
    ctx.close()
    gg = theta.grad.tolist()
    return dict(sample=f"{n}x{n}, {steps} steps, adjoint128 parameters, oracle FP64 direct solves",
                oracle_grad=list(g), gpu_grad=gg, oracle_loss=L, gpu_loss=float(Lg.detach()),
                rel_err=[abs(a - b) / abs(b) for a, b in zip(gg, g)], oracle_s=cpu_s, cores=1)


def oracle_exact(cfg, n, st0, taus):
    """CPU leg: the oracle's exact solve (one 2x2 solve per Fourier mode) of the
    first step at each tau: {tau: (phi, mu, Phi)}."""
    from oracle import potential as pot, solvers
    from oracle.systems import Params
    phi0, Phi0 = st0["phi"][0], st0["Phi_v"]
    Kh, Mh = solvers.p1_symbols(n)
    Mx = lambda v: np.real(np.fft.ifft2(Mh * np.fft.fft2(v.reshape(n, n)))).ravel()
    fp, fv = pot.dfdphi_bin(phi0, Phi0), pot.dfdPhi_bin(phi0, Phi0)
    out = {}
    for tau in taus:
        prm = Params(eps=cfg["eps"], tau=tau, mobility=cfg["mobility"], evap_rate=cfg["evap_rate"])
        ph, mu = solvers.fft_ch_solve(n, prm, Mx(phi0), -(prm.tau * prm.gamma / prm.beta) * Mx(fp))
        Ph = solvers.fft_ac_solve(n, prm, Mx(Phi0) - prm.tau * prm.gamma_v * Mx(fv))
        out[tau] = (ph, mu, Ph)
    return out


def oracle_errors(cfg, n, st0, sweep, sweep_fields):
    """CPU leg: the oracle's exact solve of each swept step (convection-free
    periodic systems, one 2x2 solve per Fourier mode) and the relative error
    of the GPU fields against it."""
    from oracle import potential as pot, solvers
    from oracle.systems import Params
    phi0, Phi0 = st0["phi"][0], st0["Phi_v"]
    Kh, Mh = solvers.p1_symbols(n)
    Mx = lambda v: np.real(np.fft.ifft2(Mh * np.fft.fft2(v.reshape(n, n)))).ravel()
    fp, fv = pot.dfdphi_bin(phi0, Phi0), pot.dfdPhi_bin(phi0, Phi0)
    for row in sweep:
        prm = Params(eps=cfg["eps"], tau=row["tau"], mobility=cfg["mobility"], evap_rate=cfg["evap_rate"])
        t0 = time.perf_counter()
        ph, mu = solvers.fft_ch_solve(n, prm, Mx(phi0), -(prm.tau * prm.gamma / prm.beta) * Mx(fp))
        Ph = solvers.fft_ac_solve(n, prm, Mx(Phi0) - prm.tau * prm.gamma_v * Mx(fv))
        row["oracle_ms"] = (time.perf_counter() - t0) * 1e3
        # condition number of the CH block from its per-mode symbols: the forward
        # error of a solve stopped at true residual rtol is bounded by kappa rtol
        tg, cc = prm.tau * prm.gamma, prm.tau * prm.gamma / prm.beta
        m_, k_ = Mh.ravel(), Kh.ravel()
        tr, det = m_ - cc * m_, -cc * m_ * m_ - (tg * k_) ** 2
        disc = np.sqrt(np.maximum(tr * tr / 4 - det, 0.0))
        ev = np.abs(np.concatenate([tr / 2 + disc, tr / 2 - disc]))
        row["kappa_ch"] = float(ev.max() / ev.min())
        row["error_bound_kappa_rtol"] = row["kappa_ch"] * 1e-8
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        for name in ("fp64", "mixed"):
            g = sweep_fields[(row["tau"], name)]
            row[name].update(err_phi=rel(g["phi"], ph), err_mu=rel(g["mu"], mu), err_Phi=rel(g["Phi"], Ph))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (no sharding across GPUs); --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2501_11767_amd import chns, inputs
    cfg = inputs.CONFIGS["chac1024"]
    n = args.n
    N = n * n
    p = dict(eps=cfg["eps"], tau=args.tau, mobility=cfg["mobility"], evap_rate=cfg["evap_rate"])
    log(f"chac{n}: context")
    ctx = chns.Context(n, "ch_ac", **p)
    st0 = inputs.initial_state(n, "ch_ac", cfg["mean"], cfg["seed"])
    fields = {}

    def fresh():
        phi, Phi = dev(st0["phi"][0]), dev(st0["Phi_v"])
        mu = torch.zeros(N, dtype=torch.float64, device="cuda")
        fields.update(phi=phi, mu=mu, Phi=Phi)
        return ctx.fields(phi=[phi], mu=[mu], Phi_v=Phi)

    # seeded level-k state (inputs) and the step's outputs live in separate buffers
    f_in = fresh()
    f_out = ctx.fields(phi=[torch.empty(N, dtype=torch.float64, device="cuda")],
                       mu=[torch.empty(N, dtype=torch.float64, device="cuda")],
                       Phi_v=torch.empty(N, dtype=torch.float64, device="cuda"))
    res = {}
    forms = [f for f in args.forms.split(",") if f]
    for name, prec in (("mixed", chns.MIXED), ("fp64", chns.F64)):
        if name not in forms:
            continue
        opts = chns.default_opts(rtol=1e-8, precision=prec, restart=args.restart, **MG)
        log(f"chac{n}: {name} warmup {args.warmup} + {args.steps} timed steps")
        run_steps(ctx, chns, f_in, f_out, args.warmup, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        walls, infos = run_steps(ctx, chns, f_in, f_out, args.steps, opts)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        di, solve_ms = dof_iters(infos, N)
        d0, d1 = ctx.diagnostics(f_in), ctx.diagnostics(f_out)  # FP64 GPU reductions, outside the timing
        res[name] = dict(
            value=di / (solve_ms * 1e-3), ms_per_step=total * 1e3 / args.steps,
            ms_per_step_median=float(np.median(walls)),
            ch_iters=[i[0]["iters"] for i in infos], ac_iters=[i[1]["iters"] for i in infos],
            converged=all(i[0]["converged"] and i[1]["converged"] for i in infos),
            rel_res_ch=max(i[0]["res_true"] / i[0]["bnorm"] for i in infos),
            mass_phi_rel_change=(d1[0] - d0[0]) / d0[0], mass_Phi_v=[d0[3], d1[3]],
            energy=[d0[4], d1[4]])
    # the same steps with a cold rate predictor: chns_set_params (untimed)
    # before each step makes FGMRES forget the previous solve's reduction rate
    for name, prec in (("mixed", chns.MIXED), ("fp64", chns.F64)):
        if name not in res:
            continue
        opts = chns.default_opts(rtol=1e-8, precision=prec, restart=args.restart, **MG)
        walls = []
        for _ in range(args.steps):
            ctx.set_params(**p)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.timestep(f_in, f_out, 1, opts)
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t0) * 1e3)
        res[name]["ms_per_step_cold_predictor"] = float(np.mean(walls))
    traj = None
    if not args.no_trajectory and "mixed" in forms:
        traj = trajectory_section(chns, ctx, st0, p, args)
    kern = {}
    if not args.no_ledger and "mixed" in forms:
        log("kernels: ledger passes (the timed steps again, one kernel class per pass)")
        kern = kernel_ledger(ctx, chns, f_in, f_out, args.steps,
                             chns.default_opts(rtol=1e-8, precision=chns.MIXED, restart=args.restart, **MG),
                             args.kernel_passes)
    probe = None if args.no_copy_probe else copy_probe()

    sweep, sweep_fields = [], {}
    exact = None
    if not args.no_sweep and not args.no_cpu:
        log("cpu leg: the oracle's exact solves of the swept steps")
        exact = oracle_exact(cfg, n, st0, cfg["tau_sweep"])
    if not args.no_sweep:
        for tau in cfg["tau_sweep"]:
            log(f"sweep: tau {tau}")
            ctx.set_params(**dict(p, tau=tau))
            row = dict(tau=tau)
            for name, prec in (("fp64", chns.F64), ("mixed", chns.MIXED)):
                def timed_step(rtol):
                    opts = chns.default_opts(rtol=rtol, precision=prec, restart=args.restart, maxiter=2000,
                                             **MG)
                    ctx.timestep(f_in, f_out, 1, opts)  # warm (the rate history of this system)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    rc, inf = ctx.timestep(f_in, f_out, 1, opts)
                    torch.cuda.synchronize()
                    return (time.perf_counter() - t0) * 1e3, inf
                wall, inf = timed_step(1e-8)
                sweep_fields[(tau, name)] = {"phi": f_out._keep[0][0].cpu().numpy(),
                                             "mu": f_out._keep[1][0].cpu().numpy(),
                                             "Phi": f_out._keep[2].cpu().numpy()}
                row[name] = dict(ms_to_rres_1e8=wall, ch_iters=inf[0]["iters"], ac_iters=inf[1]["iters"],
                                 converged=bool(inf[0]["converged"] and inf[1]["converged"]))
                if exact is not None:
                    # time to a forward error <= 1e-8 in every field: the loosest
                    # tolerance of 1e-8 ... 1e-12 whose result meets it
                    ex = exact[tau]
                    for rtol in (1e-8, 1e-9, 1e-10, 1e-11, 1e-12):
                        w, inf_r = timed_step(rtol)
                        got = (f_out._keep[0][0].cpu().numpy(), f_out._keep[1][0].cpu().numpy(),
                               f_out._keep[2].cpu().numpy())
                        err = max(float(np.linalg.norm(g - e) / np.linalg.norm(e)) for g, e in zip(got, ex))
                        if err <= 1e-8:
                            row[name].update(ms_to_err_1e8=w, rtol_for_err_1e8=rtol, err_at_that_rtol=err,
                                             ch_iters_for_err_1e8=inf_r[0]["iters"])
                            break
                    else:
                        row[name].update(ms_to_err_1e8=None, rtol_for_err_1e8=None)
            sweep.append(row)
        ctx.set_params(**p)
    if args.dry_steps > 0:
        log(f"dry256: {args.dry_steps} steps")
    dry = dry_section(chns, args.dry_steps) if args.dry_steps > 0 else None
    bat = batch_section(chns, args.batch_steps) if args.batch_steps > 0 else None
    box = box_section(chns, args.box_steps, BOX_RESTART) if args.box_steps > 0 else None
    quad = quad_section(chns, args.quad_steps) if args.quad_steps > 0 else None
    qbox = quadbox_section(chns, args.quad_steps) if args.quad_steps > 0 else None
    cube = cube_section(chns, args.cube_steps, CUBE_RESTART) if args.cube_steps > 0 else None
    adj = None if args.no_adjoint else adjoint_section(chns)
    cpu = None
    if not args.no_cpu:
        log("cpu baseline: oracle on the host")
        cpu = cpu_baseline(cfg, n, args.tau)
        if sweep:
            oracle_errors(cfg, n, st0, sweep, sweep_fields)
        if adj is not None:
            log("cpu leg: oracle adjoint on a bounded sample")
            from threadpoolctl import threadpool_limits
            with threadpool_limits(1):
                adj["cpu_reference"] = cpu_adjoint_reference(chns)

    # roofline kernel: the ledger class with the largest time per step (the
    # finest-level multigrid passes, four modes of one kernel); the others'
    # figures are in "kernels"
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"]) if kern else None
    kd = kern.get(dom) if dom else None
    # the value is the mixed form's unless only FP64 ran (--forms "" for runs of the other sections only)
    head = res.get("mixed") or res.get("fp64") or {"value": None, "ms_per_step": None}
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "DOF·iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (FGMRES) + f32 (multigrid)",
        "data": "synthetic",
        "config": {"workload": f"chac{n}: coupled CH + AC step, periodic {n}x{n} P1 ({N} nodes, "
                               f"{3 * N} unknowns), eps {cfg['eps']}, tau {args.tau}, FGMRES({args.restart}) "
                               f"rtol 1e-8, V({MG['mg_pre']},{MG['mg_post']}) block preconditioner (hierarchies cut "
                               f"at rho <= {MG['mg_rho_cut']}, {MG['mg_coarse']} coarse steps)",
                   "n": n, "tau": args.tau, "restart": args.restart,
                   "baseline_config": "mixed-precision form vs FP64, 1024x1024 P1 CH + AC, eps 0.005, tau swept "
                                      "over 1e-5 ... 1e-2, FP32 preconditioner sweeps in FP64 refinement to 1e-8",
                   "as_run": f"timed: {args.steps} steps at tau {args.tau}, each re-solving the seeded first step "
                             "(the explicit potential term makes longer runs at this tau blow up: "
                             "tests/test_oracle_step.py::test_explicit_potential_limits_the_time_step), with the "
                             "solver's rate predictor warm and (ms_per_step_cold_predictor) cold; a real 10-step "
                             "trajectory at tau 1e-5 ('trajectory'); one step per swept tau with the error against "
                             "the exact Fourier solve and the time to a forward error <= 1e-8 ('sweep')"},
        "roofline": None if kd is None else {
            "bound": "hbm", "kernel": dom, "achieved": kd["gbs"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": kd["frac"], "traffic": TRAFFIC.get(dom),
            "bytes_per_launch": kd["bytes_per_launch"], "us_per_launch": kd["us_per_launch"],
            "launches": kd["launches"],
            "frac_of_streaming_probe": None if probe is None else kd["gbs"] / probe["gbs"]},
        "cpu_baseline": cpu,
        "mixed": res.get("mixed"),
        "fp64": res.get("fp64"),
        "kernels": {name: dict(f, frac_of_streaming_probe=None if probe is None else f["gbs"] / probe["gbs"])
                    for name, f in kern.items()},
        "copy_probe": probe,
        "sweep": sweep,
        "trajectory": traj,
        "dry256": dry,
        "batch64": bat,
        "box10": box,
        "quad256": quad,
        "quadbox": qbox,
        "cube40": cube,
        "adjoint128": adj,
    }
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
