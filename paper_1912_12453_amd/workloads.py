"""Seeded synthetic workloads: geometry indicators, parameters and fields.

This module only generates inputs.  It holds none of the method's arithmetic
(no residual, no quadrature, no solver); the CPU oracle and the GPU library
both receive the arrays it returns.  Random draws use numpy's PCG64
``default_rng(seed)``; fields are returned in the node order of the mesh they
are evaluated on (node-major, 6 doubles per node: phi, mu, u, v, w, p).

The paper's experiments (Sec. 5) need literature and experimental data that
are not available; these workloads take their shapes and parameter ranges
instead:

* ``drop16``      -- one Crank-Nicolson step on a uniform 16^3 mesh, heavy drop
                     (density ratio 10) in a lighter fluid.
* ``bubble_l9``   -- rising-bubble geometry (radius 0.15 at (0.5,0.3,0.5),
                     Cn 0.005) refined to level 9 near the interface, density
                     ratio 1000, viscosity ratio 100; random velocity.
* ``rt_l10``      -- Rayleigh-Taylor interface z = 2 + 0.05 cos(2 pi x)
                     cos(2 pi y) in a 1x1x4 brick, Atwood 0.5, level 10.
* ``serving``     -- droplet/bubble requests with 1-4 drops of random radius,
                     max level 6..9, density ratio 2..1000.
"""
from dataclasses import dataclass, field, replace
import math

import numpy as np

SQRT2 = math.sqrt(2.0)


# --------------------------------------------------------------- geometry ---
def sphere_phi(centre, radius, Cn, inside=+1.0):
    """phi0(x) = inside * tanh((radius - |x - c|) / (sqrt(2) Cn)): the
    equilibrium tanh profile, +inside within the sphere."""
    c = np.asarray(centre, dtype=np.float64)

    def f(xyz):
        d = np.sqrt(((xyz - c) ** 2).sum(axis=1))
        return inside * np.tanh((radius - d) / (SQRT2 * Cn))
    return f


def drops_phi(drops, Cn, inside=+1.0):
    """Union of several drops: the pointwise maximum of inside*profile, then the
    sign convention applied (inside=-1 gives light bubbles)."""
    cs = [np.asarray(c, dtype=np.float64) for c, _ in drops]
    rs = [float(r) for _, r in drops]

    def f(xyz):
        best = None
        for c, r in zip(cs, rs):
            v = np.tanh((r - np.sqrt(((xyz - c) ** 2).sum(axis=1))) / (SQRT2 * Cn))
            best = v if best is None else np.maximum(best, v)
        return inside * best
    return f


def rt_phi(Cn, z0=2.0, amp=0.05):
    """phi0 = tanh((z_int(x,y) - z)/(sqrt(2) Cn)), z_int = z0 + amp cos(2 pi x) cos(2 pi y):
    +1 below the interface."""
    def f(xyz):
        zi = z0 + amp * np.cos(2 * np.pi * xyz[:, 0]) * np.cos(2 * np.pi * xyz[:, 1])
        return np.tanh((zi - xyz[:, 2]) / (SQRT2 * Cn))
    return f


# ------------------------------------------------------------- parameters ---
@dataclass
class Physics:
    Cn: float
    Pe: float
    Re: float
    We: float
    Fr: float
    rho_minus: float     # rho_- / rho_+ (rho(+1) = 1, rho(-1) = rho_minus)
    eta_minus: float     # eta_- / eta_+
    dt: float
    g: tuple = (0.0, -1.0, 0.0)
    C_I: float = 6.0
    flux_mode: int = 0


@dataclass
class MeshSpec:
    trees: tuple = (1, 1, 1)
    level_min: int = 4
    level_max: int = 4
    phi0: object = None
    band: float = 0.9


@dataclass
class Workload:
    name: str
    mesh: MeshSpec
    physics: Physics
    steps: int = 1
    seeds: dict = field(default_factory=dict)
    description: str = ""


def drop16(level=4):
    """Uniform level-4 (16^3) unit cube, 4913 nodes; heavy drop of radius 0.25."""
    Cn = 0.04
    return Workload(
        name=f"drop{2 ** level}",
        mesh=MeshSpec((1, 1, 1), level, level, None, 0.9),
        physics=Physics(Cn=Cn, Pe=1.0 / Cn, Re=100.0, We=10.0, Fr=1.0, rho_minus=0.1,
                        eta_minus=0.1, dt=1e-3),
        steps=1, seeds={"perturb": 0},
        description=f"uniform {2 ** level}^3 Q1 mesh, heavy drop r=0.25, density/viscosity ratio 10")


def bubble(level_max=9, level_min=4):
    """Rising-bubble mesh: level_max within |phi0| < 0.9, level_min elsewhere."""
    Cn = 0.005
    return Workload(
        name=f"bubble_l{level_max}",
        mesh=MeshSpec((1, 1, 1), level_min, level_max,
                      sphere_phi((0.5, 0.3, 0.5), 0.15, Cn, inside=-1.0), 0.9),
        physics=Physics(Cn=Cn, Pe=1.0 / (3 * Cn * Cn), Re=35.0, We=10.0, Fr=1.0,
                        rho_minus=1e-3, eta_minus=1e-2, dt=5e-4),
        steps=10, seeds={"velocity": 1, "perturb": 2, "direction": 3},
        description=f"bubble r=0.15 Cn=0.005 refined to level {level_max}, density ratio 1000, "
                    "viscosity ratio 100")


def rt(level_max=10, level_min=4):
    """Rayleigh-Taylor brick 1x1x4, z vertical, Atwood 0.5."""
    Cn = 0.0025
    return Workload(
        name=f"rt_l{level_max}",
        mesh=MeshSpec((1, 1, 4), level_min, level_max, rt_phi(Cn), 0.9),
        physics=Physics(Cn=Cn, Pe=1.0 / (3 * Cn * Cn), Re=1000.0, We=1000.0, Fr=1.0,
                        rho_minus=3.0, eta_minus=1.0, dt=2.5e-4, g=(0.0, 0.0, -1.0)),
        steps=20, seeds={"direction": 5},
        description=f"Rayleigh-Taylor 1x1x4 brick refined to level {level_max}, Atwood 0.5")


# ----------------------------------------------------------------- fields ---
def node_coordinates(nodes_int, level_max):
    """Physical coordinates of integer node coordinates (2^level_max units)."""
    return np.asarray(nodes_int, dtype=np.float64) * 2.0 ** (-level_max)


def initial_state(xyz, phi0, bflags=None, velocity_sigma=0.0, phi_noise=0.0, seed=0,
                  velocity_seed=None):
    """U^0: phi = phi0(x) (+ uniform noise), mu = phi^3 - phi (the bulk chemical
    potential of the profile), v = 0 or N(0, sigma^2) (zero on boundary nodes),
    p = 0."""
    n = xyz.shape[0]
    U = np.zeros((n, 6))
    phi = phi0(xyz) if phi0 is not None else np.ones(n)
    if phi_noise > 0:
        phi = phi + np.random.default_rng(seed).uniform(-phi_noise, phi_noise, n)
    U[:, 0] = phi
    U[:, 1] = phi ** 3 - phi
    if velocity_sigma > 0:
        rng = np.random.default_rng(seed if velocity_seed is None else velocity_seed)
        U[:, 2:5] = rng.normal(0.0, velocity_sigma, (n, 3))
        if bflags is not None:
            U[(np.asarray(bflags) & 1) != 0, 2:5] = 0.0
    return U


def perturbed(U, sigma, seed):
    """U + N(0, sigma^2) on every entry (a non-converged iterate U^{k+1})."""
    return U + np.random.default_rng(seed).normal(0.0, sigma, U.shape)


def direction(n, seed, dtype=np.float64):
    """A Krylov-like direction dU ~ N(0, 1), node-major 6 fields."""
    return np.random.default_rng(seed).normal(0.0, 1.0, (n, 6)).astype(dtype)


def random_leaves(trees, level_max, seed, p_split=0.4, level_min=0):
    """A random (unbalanced) octree: each octant below level_max splits with
    probability p_split (always below level_min).  Returns (x,y,z,level) rows."""
    rng = np.random.default_rng(seed)
    out = []
    stack = []
    for k in range(trees[2]):
        for j in range(trees[1]):
            for i in range(trees[0]):
                stack.append((i << level_max, j << level_max, k << level_max, 0))
    while stack:
        x, y, z, l = stack.pop()
        if l < level_max and (l < level_min or rng.random() < p_split):
            h = 1 << (level_max - l - 1)
            for c in range(8):
                stack.append((x + (h if c & 1 else 0), y + (h if c & 2 else 0),
                              z + (h if c & 4 else 0), l + 1))
        else:
            out.append((x, y, z, l))
    return np.array(out, dtype=np.int32)


# ----------------------------------------------------------------- serving ---
@dataclass
class Request:
    rid: int
    arrival_s: float
    workload: Workload
    kind: str


def serving_stream(n_requests=64, rate_hz=20.0, seed=4, level_range=(6, 9), steps=10):
    """Independent droplet/bubble problems arriving as a Poisson process."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    Cn = 0.01
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        nd = int(rng.integers(1, 5))
        drops = []
        tries = 0
        while len(drops) < nd and tries < 1000:
            tries += 1
            r = rng.uniform(0.08, 0.2)
            c = rng.uniform(r + 0.05, 1 - r - 0.05, 3)
            if all(np.linalg.norm(c - c2) > r + r2 + 4 * SQRT2 * Cn for c2, r2 in drops):
                drops.append((c, r))
        bubble_kind = bool(rng.integers(0, 2))
        ratio = rng.uniform(2.0, 1000.0)
        visc = rng.uniform(1.0, 100.0)
        lmax = int(rng.integers(level_range[0], level_range[1] + 1))
        # the drop phase is phi = -1 in both cases; rho(+1) = 1 is the outer fluid
        inside = -1.0
        rho_minus = (1.0 / ratio) if bubble_kind else ratio
        eta_minus = (1.0 / visc) if bubble_kind else visc
        wl = Workload(
            name=f"req{rid}",
            mesh=MeshSpec((1, 1, 1), 4, lmax, drops_phi(drops, Cn, inside), 0.9),
            physics=Physics(Cn=Cn, Pe=1.0 / (3 * Cn * Cn), Re=35.0, We=10.0, Fr=1.0,
                            rho_minus=rho_minus, eta_minus=eta_minus, dt=5e-4),
            steps=steps, seeds={},
            description=f"{nd} {'bubbles' if bubble_kind else 'droplets'} level {lmax}")
        reqs.append(Request(rid, t, wl, "bubble" if bubble_kind else "droplet"))
    return reqs


def with_physics(w: Workload, **kw):
    return replace(w, physics=replace(w.physics, **kw))


def random_state(n, seed, phi_range=1.1, mu_sigma=0.5, v_sigma=0.3, p_sigma=1.0, step=0.05):
    """A generic non-converged pair (U^{k+1}, U^k) for parity checks: phi ~
    U(-phi_range, phi_range) (so some values need the pull-back), mu, v, p
    normal; U^{k+1} = U^k + N(0, step^2)."""
    rng = np.random.default_rng(seed)
    U0 = np.zeros((n, 6))
    U0[:, 0] = rng.uniform(-phi_range, phi_range, n)
    U0[:, 1] = rng.normal(0, mu_sigma, n)
    U0[:, 2:5] = rng.normal(0, v_sigma, (n, 3))
    U0[:, 5] = rng.normal(0, p_sigma, n)
    U1 = U0 + rng.normal(0, step, U0.shape)
    return U1, U0


def moderate_physics(**kw):
    """Parameters of order one for parity checks on random states."""
    base = dict(Cn=0.3, Pe=2.0, Re=7.0, We=3.0, Fr=1.5, rho_minus=0.25, eta_minus=0.4, dt=0.05,
                g=(0.0, -1.0, 0.0))
    base.update(kw)
    return Physics(**base)


def bubble_state(xyz, bflags, w, seeds=None):
    """The bubble workload's fields: phi0 profile, mu = phi^3 - phi, v ~ N(0, 0.01^2)
    (zero on the boundary), p = 0 as U^k; U^{k+1} = U^k + N(0, 1e-3^2)."""
    seeds = seeds or w.seeds
    U0 = initial_state(xyz, w.mesh.phi0, bflags, velocity_sigma=0.01,
                       velocity_seed=seeds.get("velocity", 1))
    U1 = perturbed(U0, 1e-3, seeds.get("perturb", 2))
    return U1, U0


def by_name(name):
    """The workload called bubble_l<L>, rt_l<L> or drop<2^L>."""
    if name.startswith("bubble_l"):
        return bubble(level_max=int(name[len("bubble_l"):]))
    if name.startswith("rt_l"):
        return rt(level_max=int(name[len("rt_l"):]))
    if name.startswith("drop"):
        side = int(name[len("drop"):])
        level = side.bit_length() - 1
        if side != 1 << level:
            raise ValueError(f"drop side {side} is not a power of two")
        return drop16(level)
    raise ValueError(f"unknown workload {name}")


def state_for(w, xyz, bflags):
    """(U^{k+1}, U^k) of a named workload on the nodes xyz: the bubble fields for
    bubble meshes, else phi0 with 1e-3 noise and a 1e-3 perturbation."""
    if w.name.startswith("bubble"):
        return bubble_state(xyz, bflags, w)
    U0 = initial_state(xyz, w.mesh.phi0, bflags, phi_noise=1e-3, seed=0)
    return perturbed(U0, 1e-3, w.seeds.get("perturb", 2)), U0
