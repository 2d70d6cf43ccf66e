"""Seeded synthetic inputs shared by the HIP path, its tests and the CPU oracle.

This module holds no arithmetic of the method itself: it only draws the initial
fields (uniform noise about a mean, a layered vapour field, a divergence-free
random velocity from a stream function) and names the workload parameters.
Both the oracle and the GPU path receive identical arrays from here.

Numbering convention (a stated interface, used by both sides): on the periodic
unit square with n cells per side, vertex (i, j) has id ``i + n*j`` and sits at
``(i/n, j/n)``.  Quadratic (P2) velocity nodes are the n*n vertices, then the
midpoints of the horizontal edges ``(i,j)-(i+1,j)``, then of the vertical edges
``(i,j)-(i,j+1)``, then of the diagonal edges ``(i,j)-(i+1,j+1)``; each group is
numbered ``i + n*j``.

The paper's initial data (section "Numerical results", figure of the initial
condition) is a polymer/NFA/solvent film with uniform +-0.01 fluctuations; the
workloads below keep that noise model on a periodic box.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 20250117


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def vertex_coords(n: int) -> np.ndarray:
    """(n*n, 2) coordinates of the P1 nodes in id order."""
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([i.ravel() / n, j.ravel() / n], axis=1)


def p2_coords(n: int) -> np.ndarray:
    """(4*n*n, 2) coordinates of the P2 nodes in id order (see module doc)."""
    v = vertex_coords(n)
    h = 1.0 / n
    return np.concatenate(
        [v, v + [0.5 * h, 0.0], v + [0.0, 0.5 * h], v + [0.5 * h, 0.5 * h]], axis=0
    )


def noisy_field(n: int, mean: float, amp: float, seed: int) -> np.ndarray:
    """mean + amp * U(-1, 1) at every vertex."""
    return mean + amp * rng(seed).uniform(-1.0, 1.0, size=n * n)


def vapour_layer(n: int) -> np.ndarray:
    """Phi_v^0 = sin^2(pi y): liquid at y = 0 (= 1 by periodicity), vapour at y = 1/2."""
    y = vertex_coords(n)[:, 1]
    return np.sin(np.pi * y) ** 2


def stream_velocity(n: int, seed: int, modes: int = 16, amp: float = 0.01) -> np.ndarray:
    """Divergence-free velocity v = (d psi/dy, -d psi/dx) at the P2 nodes.

    psi = sum_m amp * sin(2 pi k_m . x + theta_m), k_m uniform on {-4..4}^2 minus 0,
    theta_m ~ U(0, 2 pi).  Returns (2, 4*n*n): x components then y components.
    """
    g = rng(seed)
    ks = []
    while len(ks) < modes:
        k = g.integers(-4, 5, size=2)
        if k[0] != 0 or k[1] != 0:
            ks.append(k)
    ks = np.array(ks, dtype=np.float64)
    th = g.uniform(0.0, 2.0 * np.pi, size=modes)
    xy = p2_coords(n)
    arg = 2.0 * np.pi * (xy @ ks.T) + th[None, :]
    c = amp * np.cos(arg) * 2.0 * np.pi
    vx = c @ ks[:, 1]
    vy = -(c @ ks[:, 0])
    return np.stack([vx, vy], axis=0)


def box_vertex_coords(n: int, length: float) -> np.ndarray:
    """((n+1)^2, 2) coordinates of the vertices of the closed square [0, L]^2
    with n cells per side: vertex (i, j) has id ``i + (n+1)*j`` and sits at
    ``(i L/n, j L/n)``."""
    m = n + 1
    j, i = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    return np.stack([i.ravel(), j.ravel()], axis=1) * (length / n)


def box_p2_coords(n: int, length: float) -> np.ndarray:
    """(4N, 2), N = (n+1)^2: coordinates of the P2 ids on the closed square:
    the vertices, then the midpoints of the edges (i,j)-(i+1,j), (i,j)-(i,j+1)
    and (i,j)-(i+1,j+1), each block numbered i + (n+1)*j (ids with i = n in the
    first and third edge block or j = n in the second and third belong to no
    edge)."""
    v = box_vertex_coords(n, length)
    h = length / n
    return np.concatenate([v, v + [0.5 * h, 0.0], v + [0.0, 0.5 * h], v + [0.5 * h, 0.5 * h]], axis=0)


def box_p2_unused(n: int) -> np.ndarray:
    """(4N,) True for the P2 ids of the closed square that belong to no edge."""
    m = n + 1
    j, i = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    i, j = i.ravel(), j.ravel()
    return np.concatenate([np.zeros(m * m, bool), i == n, j == n, (i == n) | (j == n)])


def box_p2_wall(n: int) -> np.ndarray:
    """(4N,) True for the P2 ids on the walls of the closed square: wall
    vertices, edges of the bottom and top walls, edges of the side walls."""
    m = n + 1
    j, i = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    i, j = i.ravel(), j.ravel()
    side, tb = (i == 0) | (i == n), (j == 0) | (j == n)
    return np.concatenate([side | tb, tb & (i < n), side & (j < n), np.zeros(m * m, bool)])


def box_stream_velocity(n: int, length: float, seed: int, amp: float = 0.01) -> np.ndarray:
    """Divergence-free velocity (d psi/dy, -d psi/dx) at the P2 ids of the
    closed square that vanishes with its stream function on the walls:
    psi = amp S(x) S(y) (1 + 0.3 sin(2 pi x/L + t1) sin(2 pi y/L + t2)),
    S(u) = sin^2(pi u/L), phases t1, t2 ~ U(0, 2 pi).  Exactly zero on the
    walls and at the unused ids.  Returns (2, 4N)."""
    t1, t2 = rng(seed).uniform(0.0, 2.0 * np.pi, size=2)
    xy = box_p2_coords(n, length)
    x, y = xy[:, 0], xy[:, 1]
    k, q = np.pi / length, 2.0 * np.pi / length
    S = lambda u: np.sin(k * u) ** 2
    dS = lambda u: 2.0 * k * np.sin(k * u) * np.cos(k * u)
    g = 1.0 + 0.3 * np.sin(q * x + t1) * np.sin(q * y + t2)
    gx = 0.3 * q * np.cos(q * x + t1) * np.sin(q * y + t2)
    gy = 0.3 * q * np.sin(q * x + t1) * np.cos(q * y + t2)
    psi_x = amp * (dS(x) * S(y) * g + S(x) * S(y) * gx)
    psi_y = amp * (S(x) * dS(y) * g + S(x) * S(y) * gy)
    vel = np.stack([psi_y, -psi_x], axis=0)
    vel[:, box_p2_unused(n) | box_p2_wall(n)] = 0.0
    return vel


def box_state(n: int, length: float, model: str, mean: float, seed: int, film: float = 0.5):
    """Initial fields on the closed square after the paper's two-dimensional
    set-up (section "Numerical results", figure of the initial condition): a
    film on the substrate y <= film * L, vapour field 0, under the ambient air
    (vapour field 1).  Binary models: the phase at mean + U(-0.01, 0.01) in the
    film, 0 above.  Ternary (solvent eliminated, no air): polymer and NFA at
    mean +- 0.01 in the film, 0 above (pure solvent).  Quaternary (air
    eliminated): polymer and NFA at mean, solvent at 1 - 2 mean (each +- 0.01)
    in the film, all three 0 above (pure air).  The flow models start from
    box_stream_velocity and p = 0.  Keys as initial_state."""
    y = box_vertex_coords(n, length)[:, 1]
    below = y <= film * length
    kids = np.random.SeedSequence(seed).spawn(4)
    seeds = [int(k.generate_state(1)[0]) for k in kids]
    noise = lambda i: rng(seeds[i]).uniform(-1.0, 1.0, size=y.size)
    Phi_v = np.where(below, 0.0, 1.0) if model != "ch" else None
    if model in ("ch", "ch_ac"):
        return dict(phi=[np.where(below, mean + 0.01 * noise(0), 0.0)], Phi_v=Phi_v, vel=None, p=None)
    if model == "ternary":
        means = (mean, mean)
    elif model == "quaternary":
        means = (mean, mean, 1.0 - 2.0 * mean)
    else:
        raise ValueError(model)
    phi = [np.where(below, means[i] + 0.01 * noise(i), 0.0) for i in range(len(means))]
    vel = box_stream_velocity(n, length, seeds[3])
    return dict(phi=phi, Phi_v=Phi_v, vel=vel, p=np.zeros(y.size))


def cube_vertex_coords(n: int, length: float = 1.0) -> np.ndarray:
    """(n^3, 3) coordinates of the periodic cube's vertices, id i + n j + n^2 k."""
    k, j, i = np.unravel_index(np.arange(n ** 3), (n, n, n))
    return np.stack([i, j, k], 1) * (length / n)


def cube_state(n: int, model: str, mean: float, seed: int, length: float = 1.0):
    """Initial fields of the binary models on the periodic cube: the phase at
    mean + U(-0.01, 0.01) at every vertex; the vapour field (CH + AC) a layer
    sin^2(pi z / L), liquid at z = 0 and vapour at z = L/2.  Keys as
    initial_state."""
    if model not in ("ch", "ch_ac"):
        raise ValueError(model)
    phi = mean + 0.01 * rng(seed).uniform(-1.0, 1.0, size=n ** 3)
    z = cube_vertex_coords(n, length)[:, 2]
    Phi_v = np.sin(np.pi * z / length) ** 2 if model == "ch_ac" else None
    return dict(phi=[phi], Phi_v=Phi_v, vel=None, p=None)


def cube_box_state(n: int, length: float, model: str, mean: float, seed: int, film: float = 0.5):
    """Initial fields of the binary models on the closed cube [0, L]^3 ((n+1)^3
    vertices), the three-dimensional form of box_state: a film z <= film * L at
    mean + U(-0.01, 0.01) with vapour field 0, air above (phase 0, vapour
    field 1).  Keys as initial_state."""
    if model not in ("ch", "ch_ac"):
        raise ValueError(model)
    z = cube_vertex_coords(n + 1, length * (n + 1) / n)[:, 2]
    below = z <= film * length
    phi = np.where(below, mean + 0.01 * rng(seed).uniform(-1.0, 1.0, size=z.size), 0.0)
    Phi_v = np.where(below, 0.0, 1.0) if model == "ch_ac" else None
    return dict(phi=[phi], Phi_v=Phi_v, vel=None, p=None)


def log_uniform(g: np.random.Generator, lo: float, hi: float) -> float:
    return float(np.exp(g.uniform(np.log(lo), np.log(hi))))


# Workloads.  "binary" = one Cahn-Hilliard phase with the double-well / mixing
# potential; "ternary" = polymer and NFA phases (solvent eliminated) with the
# fitted quartic potential, plus the vapour field and the Oseen step;
# "quaternary" = polymer, NFA and solvent phases with the air eliminated.
CONFIGS = {
    "ch32": dict(n=32, model="ch", eps=0.02, tau=1e-3, mobility=1.0, evap_rate=0.0,
                 viscosity=1.0, steps=1, mean=0.5, seed=BASE_SEED + 0),
    "dry256": dict(n=256, model="ternary", eps=0.01, tau=5e-4, mobility=1.0, evap_rate=0.1,
                   viscosity=1.0, steps=20, mean=0.3, seed=BASE_SEED + 1),
    "chac1024": dict(n=1024, model="ch_ac", eps=0.005, tau=1e-4, mobility=1.0, evap_rate=0.1,
                     viscosity=1.0, steps=1, mean=0.4, seed=BASE_SEED + 2,
                     tau_sweep=(1e-5, 1e-4, 1e-3, 1e-2)),
    # the paper's closed domain and two-phase set-up (section "Evaporation of
    # solvent" with its two-dimensional appendix): 10 x 10 square with no-flux
    # boundaries, a film at 1 +- 0.01 under air, beta = 0.1, gamma = gamma_v = 1,
    # tau = 1e-4; 128 cells per side (the paper takes 100) so that the
    # multigrid hierarchy halves down to 4
    "box10": dict(n=128, length=10.0, model="ch_ac", eps=0.1 ** 0.5, tau=1e-4, mobility=1.0,
                  evap_rate=1.0, viscosity=1.0, steps=1, mean=1.0, seed=BASE_SEED + 5),
    # the paper's full system (polymer, NFA, solvent, air eliminated) with its
    # per-phase gradient coefficients beta_p = beta_N = 1e-3, beta_s = 1e-1,
    # beta_a = beta_v = 1 scaled by eps^2 = 1e-4 onto the periodic unit square
    # (the ratios kept), tau = 1e-4, gamma = gamma_v = 1, alpha = 1e-8, a = 0.33
    "quad256": dict(n=256, model="quaternary", eps=0.01, tau=1e-4, mobility=1.0, evap_rate=1.0,
                    viscosity=1.0, alpha=1e-8, betas=(1e-7, 1e-7, 1e-5, 1e-4), steps=1, mean=0.33,
                    seed=BASE_SEED + 6),
    # the paper's full two-dimensional run (section "Numerical results", figure
    # of GMRES iterations for polymer, NFA, solvent and Navier-Stokes): the
    # closed 10 x 10 square, no-flux walls, no-slip velocity, beta_p = beta_N =
    # 1e-3, beta_s = 1e-1, beta_a = beta_v = delta_v = 1 (eps = 1, gamma_v = 1),
    # gamma = 1, alpha = 1e-8, tau = 1e-4, a = b = 0.33; 64 cells per side (the
    # paper takes 50) so that the hierarchy halves to 4
    "quadbox": dict(n=64, length=10.0, model="quaternary", eps=1.0, tau=1e-4, mobility=1.0, evap_rate=1.0,
                    viscosity=1.0, alpha=1e-8, betas=(1e-3, 1e-3, 1e-1, 1.0), steps=1, mean=0.33,
                    seed=BASE_SEED + 7),
    # the paper's three-dimensional runs on a uniform 40 x 40 x 40 grid (section
    # "Numerical results", tau = 1e-4), here for the binary CH + AC model on the
    # periodic unit cube (Kuhn tetrahedra; levels 40, 20, 10, 5), a film mean of
    # 0.4, eps = 0.05 (2 cells of the mesh); 128 cells per side as the larger size
    "cube40": dict(n=40, model="ch_ac", eps=0.05, tau=1e-4, mobility=1.0, evap_rate=0.1,
                   viscosity=1.0, steps=1, mean=0.4, seed=BASE_SEED + 8, sizes=(40, 64, 128)),
    # the paper's three-dimensional domain: the closed 10 x 10 x 10 cube with
    # no-flux walls on its 40^3 grid, the two-phase set-up of box10 (film at
    # 1 +- 0.01 under air, beta = 0.1, gamma = gamma_v = 1, tau = 1e-4)
    "cubebox40": dict(n=40, length=10.0, model="ch_ac", eps=0.1 ** 0.5, tau=1e-4, mobility=1.0,
                      evap_rate=1.0, viscosity=1.0, steps=1, mean=1.0, seed=BASE_SEED + 9),
    "batch64": dict(instances=64, sizes=(64, 128, 256, 512), seed=BASE_SEED + 3),
    # Differentiation workload.  With the explicit potential the ternary run on
    # this mesh diverges within 6 steps at tau = 1e-3, 8 at 1e-4 and 17 at 1e-5
    # (both parameter sets); tau = 3e-6 is the largest probed step whose 50-step
    # trajectory stays bounded at theta_ref and theta0, so the run uses it.
    # mu^0 = 0 and p^0 = 0 (data, independent of theta).
    "adjoint128": dict(n=128, model="ternary", eps=0.015, tau=3e-6, mobility=2.0, evap_rate=0.2,
                       viscosity=1.0, alpha=1e-8, steps=50, checkpoint=10, mean=0.3,
                       seed=BASE_SEED + 4, theta0=(0.0125, 1.5, 0.15), tau_stated=1e-3),
}


def initial_state(n: int, model: str, mean: float, seed: int, with_velocity: bool | None = None):
    """Initial fields for a workload.  Keys: phi (list of arrays), Phi_v, vel, p.

    Each field draws from its own child stream of ``SeedSequence(seed)``.
    """
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(5 if model == "quaternary" else 4)
    seeds = [int(k.generate_state(1)[0]) for k in kids]
    flow = model in ("ternary", "quaternary")
    if model == "quaternary":
        # the paper's film (polymer and NFA at mean, solvent at 1 - 2 mean, each
        # +- 0.01) where the vapour layer is liquid (Phi_v^0 < 1/2), air (all
        # three phases 0) where it is vapour
        film = vapour_layer(n) < 0.5
        means = (mean, mean, 1.0 - 2.0 * mean)
        phi = [np.where(film, noisy_field(n, means[i], 0.01, seeds[i if i < 2 else 4]), 0.0)
               for i in range(3)]
    else:
        nphase = 2 if model == "ternary" else 1
        phi = [noisy_field(n, mean, 0.01, seeds[i]) for i in range(nphase)]
    Phi_v = vapour_layer(n) if model in ("ch_ac", "ternary", "quaternary") else None
    if with_velocity is None:
        with_velocity = flow
    vel = stream_velocity(n, seeds[2]) if with_velocity else None
    p = np.zeros(n * n) if flow else None
    return dict(phi=phi, Phi_v=Phi_v, vel=vel, p=p)


def batch_instances(count: int = 64, sizes=(64, 128, 256, 512), seed: int = BASE_SEED + 3):
    """Per-instance mesh size and parameters for the batched workload."""
    g = rng(seed)
    out = []
    for _ in range(count):
        out.append(dict(
            n=int(g.choice(sizes)),
            eps=log_uniform(g, 0.005, 0.05),
            tau=log_uniform(g, 1e-5, 1e-2),
            mobility=log_uniform(g, 0.1, 10.0),
            evap_rate=log_uniform(g, 0.01, 1.0),
            seed=int(g.integers(0, 2**31 - 1)),
        ))
    return out
