"""Seeded synthetic inputs for the metaball-coupled lattice Boltzmann step.

This module only draws numbers and lays them out; it holds none of the
method's arithmetic (no lattice tables, no body properties, no fit).  Two
helpers evaluate a metaball, only to place inputs: extent_radius (the size of
a drawn body, for placing bodies without overlap) and mi_hull (points on the
surface of a known metaball, the synthetic stand-in for the XRCT point hull
that the Metaball-Imaging fit takes as input).  Both the CPU oracle and the
HIP library read exactly what it returns, so the two sides start from
identical inputs.

A metaball body (paper section 2.1, Eq. metaballM) is a set of control points
p_i with positive weights k_i; its surface is sum_i k_i/|x - p_i|^2 = 1.  The
paper fits bodies to X-ray CT scans, which are not available, so bodies are
drawn at random: offsets p_i ~ N(0, (0.4 R)^2) per axis and k_i = R^2 u_i /
sum(u), u_i ~ U[20, 60], so that sum(k) = R^2 and the far field looks like a
sphere of radius R.  Control points are given in a body frame whose origin is
placed at ``x``; the library and the oracle each compute the true centroid
themselves.

RNG: numpy.random.Generator(PCG64(seed)); per body the draw order is n_cp,
R (only where they are random), offsets, then u.
"""
from __future__ import annotations

import copy
import dataclasses
import math
from typing import List, Optional

import numpy as np

PERIODIC_X, PERIODIC_Y, PERIODIC_Z = 1, 2, 4
BC_SBB, BC_IBB = 0, 1
STORE_F32, STORE_F16, STORE_BF16 = 0, 1, 2
MODE_FREE, MODE_KINEMATIC = 0, 1


@dataclasses.dataclass
class Particle:
    cp_xyz: np.ndarray            # (n_cp, 3) float64, body frame
    cp_k: np.ndarray              # (n_cp,)  float64, > 0
    x: np.ndarray                 # (3,) lab position of the body-frame origin
    quat: np.ndarray = dataclasses.field(default_factory=lambda: np.array([1.0, 0, 0, 0]))
    v: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    omega: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    density: float = 1.5          # absolute density (lattice units, rho0 = 1)
    mode: int = MODE_FREE         # MODE_FREE: Newton-Euler; MODE_KINEMATIC: moves with v, omega

    @property
    def n_cp(self) -> int:
        return int(self.cp_k.shape[0])

    def bounding_radius(self) -> float:
        """Radius about the body-frame origin that contains the body (C >= 1
        needs some |x - p_i|^2 <= sum k)."""
        return float(np.max(np.linalg.norm(self.cp_xyz, axis=1)) + math.sqrt(self.cp_k.sum()))


@dataclasses.dataclass
class Config:
    nx: int
    ny: int
    nz: int
    periodic: int = 0
    tau: float = 0.8
    rho0: float = 1.0
    g_fluid: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    g_particle: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    bc: int = BC_IBB
    n_sub: int = 1
    counter_force: int = 0
    quad_h: float = 0.125
    storage: int = STORE_F32
    # contact (sphero-metaball, linear spring-dashpot); contact_kn = 0 disables it
    contact_rs: float = 1.0
    contact_kn: float = 0.0
    contact_en: float = 0.5
    contact_mu: float = 0.5
    # 1: link fractions on the sphero-metaball level set f_in = c_0 (needs contact_rs > 0)
    link_c0: int = 0
    particles: List[Particle] = dataclasses.field(default_factory=list)
    name: str = ""
    steps: int = 0

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def copy(self) -> "Config":
        return copy.deepcopy(self)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_body(rng: np.random.Generator, n_cp: int, R: float):
    offsets = rng.normal(0.0, 0.4 * R, size=(n_cp, 3))
    u = rng.uniform(20.0, 60.0, size=n_cp)
    k = R * R * u / u.sum()
    return offsets.astype(np.float64), k.astype(np.float64)


# ---------------------------------------------------------------- configs
def config1(center: str = "integer", bc: int = BC_SBB, n: int = 64) -> Config:
    """64^3 periodic, tau 0.8, one fixed single-control-point body (k = 64,
    sphere of radius 8) at the box centre, body force 1e-6 along +x, 200 steps."""
    c = n / 2 if center == "integer" else n / 2 - 0.5
    p = Particle(cp_xyz=np.zeros((1, 3)), cp_k=np.array([64.0 * (n / 64) ** 2]),
                 x=np.array([c, c, c]), density=1.0, mode=MODE_KINEMATIC)
    return Config(nx=n, ny=n, nz=n, periodic=7, tau=0.8, rho0=1.0,
                  g_fluid=np.array([1e-6, 0.0, 0.0]), bc=bc, particles=[p],
                  name=f"cfg1-{n}^3-{center}", steps=200)


def config2(scale: float = 1.0, seed: int = 1, bc: int = BC_IBB) -> Config:
    """128x128x384 walled box, tau 0.6, one free 8-control-point body (R = 10,
    density ratio 1.5), gravity 2e-5 along -z, 2000 steps.  ``scale`` < 1
    shrinks box and body together for oracle-sized runs."""
    rng = _rng(seed)
    R = 10.0 * scale
    off, k = random_body(rng, 8, R)
    nx, ny, nz = int(round(128 * scale)), int(round(128 * scale)), int(round(384 * scale))
    p = Particle(cp_xyz=off, cp_k=k, x=np.array([nx / 2, ny / 2, 326.0 * scale]), density=1.5)
    return Config(nx=nx, ny=ny, nz=nz, periodic=0, tau=0.6, rho0=1.0,
                  g_particle=np.array([0.0, 0.0, -2e-5]), bc=bc, particles=[p],
                  name=f"cfg2-{nx}x{ny}x{nz}", steps=2000)


def config3(scale: float = 1.0, storage: int = STORE_F16, bc: int = BC_IBB) -> Config:
    """160x160x640 walled box, tau 0.6, two bodies (6 control points seed 2
    leading at z = 544, 12 control points seed 3 at z = 584) on the axis
    x = y = 80, density ratio 1.2, gravity 2e-5, contact on (the kissing
    stage), 5000 steps."""
    R = 10.0 * scale
    bodies = []
    for seed, n_cp, z in ((2, 6, 544.0), (3, 12, 584.0)):
        off, k = random_body(_rng(seed), n_cp, R)
        bodies.append(Particle(cp_xyz=off, cp_k=k,
                               x=np.array([80.0 * scale, 80.0 * scale, z * scale]), density=1.2))
    nx, ny, nz = int(round(160 * scale)), int(round(160 * scale)), int(round(640 * scale))
    return Config(nx=nx, ny=ny, nz=nz, periodic=0, tau=0.6, rho0=1.0,
                  g_particle=np.array([0.0, 0.0, -2e-5]), bc=bc, storage=storage,
                  particles=bodies, contact_rs=1.0, contact_kn=20.0, contact_en=0.5, contact_mu=0.5,
                  name=f"cfg3-{nx}x{ny}x{nz}", steps=5000)


def config4_case(b: int, ragged: bool = False) -> Config:
    """One case of the 64-case settling ensemble (seed 4000 + b)."""
    rng = _rng(4000 + b)
    nx = int(rng.integers(8, 17)) * 8
    ny = int(rng.integers(8, 17)) * 8
    nz = int(rng.integers(8, 33)) * 8
    if ragged:
        nx, ny, nz = nx - 3, ny - 5, nz - 1
    n_cp = int(rng.integers(4, 17))
    tau = float(rng.uniform(0.55, 1.0))
    ratio = float(rng.uniform(1.1, 2.5))
    R = 10.0 * min(nx, ny) / 128.0
    off, k = random_body(rng, n_cp, R)
    p = Particle(cp_xyz=off, cp_k=k, x=np.zeros(3), density=ratio)
    rb = p.bounding_radius()
    p.x = np.array([nx / 2, ny / 2, max(nz - rb - 8.0, nz / 2)])
    return Config(nx=nx, ny=ny, nz=nz, periodic=0, tau=tau, rho0=1.0,
                  g_particle=np.array([0.0, 0.0, -2e-5]), bc=BC_IBB, particles=[p],
                  name=f"cfg4-case{b}", steps=1000)


def config4(n_cases: int = 64) -> List[Config]:
    return [config4_case(b) for b in range(n_cases)]


def mini_ensemble(n_cases: int = 4, seed: int = 4100) -> List[Config]:
    """Small walled settling systems of different sizes (one ragged, not a
    multiple of 8), tau, density ratio and number of control points, with a
    gravity large enough that each body covers and uncovers nodes within
    tens of steps (ensemble tests)."""
    rng = _rng(seed)
    out = []
    for b in range(n_cases):
        nx, ny, nz = (int(v) for v in rng.integers(24, 41, size=3))
        nz += 16
        if b == 0:
            nx, ny, nz = 37, 29, 45
        n_cp = int(rng.integers(4, 12))
        tau = float(rng.uniform(0.55, 1.0))
        ratio = float(rng.uniform(1.1, 2.5))
        R = 0.16 * min(nx, ny)
        off, k = random_body(rng, n_cp, R)
        p = Particle(cp_xyz=off, cp_k=k, x=np.array([nx / 2 + 0.3, ny / 2 - 0.2, nz * 0.6]),
                     density=ratio, omega=np.array([0.001, 0.0, 0.002]))
        out.append(Config(nx=nx, ny=ny, nz=nz, periodic=0, tau=tau, rho0=1.0,
                          g_particle=np.array([0.0, 0.0, -4e-4]), bc=BC_IBB, particles=[p],
                          name=f"mini{b}-{nx}x{ny}x{nz}"))
    return out


def extent_radius(p: "Particle", n_dir: int = 256, dr: float = 0.25) -> float:
    """Largest distance from the control-point origin of a point with
    C >= 1 (rays in n_dir Fibonacci directions sampled every dr), at most
    the bounding radius."""
    i = np.arange(n_dir) + 0.5
    phi = np.arccos(1 - 2 * i / n_dir)
    th = np.pi * (1 + 5 ** 0.5) * i
    dirs = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], axis=1)
    r = np.arange(dr, p.bounding_radius() + dr, dr)
    pts = dirs[:, None, :] * r[None, :, None]
    d2 = ((pts[:, :, None, :] - p.cp_xyz[None, None, :, :]) ** 2).sum(-1)
    C = (p.cp_k / np.maximum(d2, 1e-300)).sum(-1)
    inside = C >= 1.0
    far = np.where(inside.any(axis=1), (inside * r[None, :]).max(axis=1), 0.0)
    return float(min(far.max() + dr, p.bounding_radius()))


def config5(n_bodies: int = 200, box: int = 256, seed: int = 5,
            max_tries: int = 2000000) -> Config:
    """256^3 periodic suspension: bodies with 6..20 control points and
    R ~ U[6, 12], placed by random sequential addition with a 1 lu gap
    between the spheres that enclose each body's C >= 1 region about its
    control-point origin (the looser bounding spheres max|p| + sqrt(sum k)
    would fill 38 % of the box, at the jamming limit of the placement),
    density ratio 1.5, gravity 2e-5, fluid counter-force, contact on;
    body-property quadrature cell 1/4."""
    rng = _rng(seed)
    bodies: List[Particle] = []
    centers = np.zeros((0, 3))
    radii = np.zeros(0)
    tries = 0
    while len(bodies) < n_bodies:
        n_cp = int(rng.integers(6, 21))
        R = float(rng.uniform(6.0, 12.0))
        off, k = random_body(rng, n_cp, R)
        p = Particle(cp_xyz=off, cp_k=k, x=np.zeros(3), density=1.5)
        re = extent_radius(p)
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("random sequential placement did not finish")
            c = rng.uniform(0.0, box, size=3)
            d = c[None, :] - centers
            d -= box * np.floor(d / box + 0.5)
            if not np.any(np.linalg.norm(d, axis=1) < re + radii + 1.0):
                break
        p.x = c
        centers = np.vstack([centers, c])
        radii = np.append(radii, re)
        bodies.append(p)
    return Config(nx=box, ny=box, nz=box, periodic=7, tau=0.6, rho0=1.0,
                  g_particle=np.array([0.0, 0.0, -2e-5]), bc=BC_IBB, counter_force=1, quad_h=0.25,
                  particles=bodies, contact_rs=1.0, contact_kn=20.0, contact_en=0.5, contact_mu=0.5,
                  name=f"cfg5-{box}^3-{n_bodies}-seed{seed}", steps=200)


# ------------------------------------------------------- validation cases
def poiseuille(tau: float, H: int = 32, g: float = 1e-6, nx: int = 4, nz: int = 4) -> Config:
    """Channel: walls normal to y (H fluid nodes), periodic in x and z,
    uniform body force g along +x, no particles."""
    return Config(nx=nx, ny=H, nz=nz, periodic=PERIODIC_X | PERIODIC_Z, tau=tau, rho0=1.0,
                  g_fluid=np.array([g, 0.0, 0.0]), bc=BC_SBB, name=f"poiseuille-H{H}-tau{tau}")


def drag_array(L: int = 32, R: float = 4.0, tau: float = 0.8, g: float = 1e-6,
               bc: int = BC_IBB) -> Config:
    """Simple-cubic array of fixed spheres: one sphere of radius R in a
    periodic L^3 cell, fluid driven by a uniform body force along +x."""
    p = Particle(cp_xyz=np.zeros((1, 3)), cp_k=np.array([R * R]),
                 x=np.array([L / 2 - 0.5, L / 2 - 0.5, L / 2 - 0.5]), density=1.0,
                 mode=MODE_KINEMATIC)
    return Config(nx=L, ny=L, nz=L, periodic=7, tau=tau, rho0=1.0,
                  g_fluid=np.array([g, 0.0, 0.0]), bc=bc, particles=[p], name=f"drag-L{L}-R{R}")


def comoving(U=(0.01, 0.005, 0.0), n: int = 32, seed: int = 11, bc: int = BC_IBB) -> Config:
    """Periodic box; one kinematic body moving with the uniform flow U."""
    off, k = random_body(_rng(seed), 6, 5.0)
    p = Particle(cp_xyz=off, cp_k=k, x=np.array([n / 2, n / 2, n / 2]), density=1.0,
                 v=np.array(U, dtype=np.float64), mode=MODE_KINEMATIC)
    return Config(nx=n, ny=n, nz=n, periodic=7, tau=0.7, rho0=1.0, bc=bc,
                  particles=[p], name=f"comoving-{n}")


def random_populations(seed: int, n_nodes: int, rho0: float = 1.0, amp: float = 1e-3):
    """Deviations f_i - w_i rho0 drawn uniformly in [-amp, amp]; shape (19, N).
    A post-collision state for one-step tests (positivity is not needed)."""
    return _rng(seed).uniform(-amp, amp, size=(19, n_nodes))


def small_settling(seed: int = 21, n: int = 40, nz: int = 64, n_cp: int = 6, R: float = 5.0,
                   bc: int = BC_IBB, ratio: float = 1.5, g: float = 2e-4) -> Config:
    """Oracle-sized settling case with a stronger gravity so that the body
    crosses lattice nodes (covering and uncovering) within tens of steps."""
    off, k = random_body(_rng(seed), n_cp, R)
    p = Particle(cp_xyz=off, cp_k=k, x=np.array([n / 2 - 0.3, n / 2 + 0.2, nz * 0.6]),
                 density=ratio, omega=np.array([0.0, 0.002, 0.001]))
    return Config(nx=n, ny=n, nz=nz, periodic=0, tau=0.7, rho0=1.0,
                  g_particle=np.array([0.0, 0.0, -g]), bc=bc, particles=[p],
                  name=f"settle-{n}x{n}x{nz}")


def two_body(seed: int = 31, n: int = 48, nz: int = 80, bc: int = BC_IBB) -> Config:
    """Two bodies on the axis of a walled box (small drafting case)."""
    bodies = []
    for j, (s, n_cp, z) in enumerate(((seed, 6, nz * 0.45), (seed + 1, 9, nz * 0.75))):
        off, k = random_body(_rng(s), n_cp, 5.0)
        bodies.append(Particle(cp_xyz=off, cp_k=k, x=np.array([n / 2 + 0.4 * j, n / 2, z]),
                               density=1.3))
    return Config(nx=n, ny=n, nz=nz, periodic=0, tau=0.65, rho0=1.0,
                  g_particle=np.array([0.0, 0.0, -1e-4]), bc=bc, particles=bodies,
                  name=f"twobody-{n}x{n}x{nz}")


def contact_pair(n: int = 40, v: float = 0.05, bc: int = BC_IBB) -> Config:
    """Two dense free spheres (R = 5) driven head-on in a periodic box, contact on."""
    bodies = []
    for j, (x, vx) in enumerate(((n / 2 - 5.2, v), (n / 2 + 5.2, -v))):
        bodies.append(Particle(cp_xyz=np.zeros((1, 3)), cp_k=np.array([25.0]),
                               x=np.array([x, n / 2 + 0.6 * j, n / 2 - 0.2]),
                               v=np.array([vx, 0.0, 0.0]), density=8.0))
    return Config(nx=n, ny=n, nz=n, periodic=7, tau=0.7, bc=bc, n_sub=10, particles=bodies,
                  contact_rs=1.0, contact_kn=20.0, contact_en=0.5, contact_mu=0.4, quad_h=0.25,
                  name=f"contact-pair-{n}")


def settle_on_floor(seed: int = 41, n: int = 32, nz: int = 28, bc: int = BC_IBB) -> Config:
    """A 7-point body dropped just above the floor of a walled box, contact on."""
    off, k = random_body(_rng(seed), 7, 5.0)
    p = Particle(cp_xyz=off, cp_k=k, x=np.zeros(3), density=2.5,
                 omega=np.array([0.0, 0.003, 0.0]), v=np.array([0.004, 0.0, -0.03]))
    rb = p.bounding_radius()
    p.x = np.array([n / 2, n / 2 + 0.4, rb + 0.2])
    return Config(nx=n, ny=n, nz=nz, periodic=PERIODIC_X | PERIODIC_Y, tau=0.8, bc=bc, n_sub=5,
                  g_particle=np.array([0.0, 0.0, -3e-3]), particles=[p], contact_rs=1.0,
                  contact_kn=20.0, contact_en=0.5, contact_mu=0.5, quad_h=0.25, name="settle-floor")


def suspension_small(n_bodies: int = 6, box: int = 48, seed: int = 51, bc: int = BC_IBB) -> Config:
    """Small periodic suspension (bodies of 4..8 points, R 3.5..5, tightly
    packed by random sequential addition), counter-force, contact on."""
    rng = _rng(seed)
    bodies, centers, radii = [], [], []
    while len(bodies) < n_bodies:
        n_cp = int(rng.integers(4, 9))
        R = float(rng.uniform(3.5, 5.0))
        off, k = random_body(rng, n_cp, R)
        p = Particle(cp_xyz=off, cp_k=k, x=np.zeros(3), density=6.0,
                     v=rng.uniform(-0.05, 0.05, 3))
        rb = p.bounding_radius()
        for _ in range(100000):
            c = rng.uniform(0.0, box, size=3)
            if all(np.linalg.norm((c - c2) - box * np.floor((c - c2) / box + 0.5)) > 0.7 * (rb + r2)
                   for c2, r2 in zip(centers, radii)):
                break
        p.x = c
        centers.append(c)
        radii.append(rb)
        bodies.append(p)
    return Config(nx=box, ny=box, nz=box, periodic=7, tau=0.7, bc=bc, n_sub=4, counter_force=1,
                  g_particle=np.array([0.0, 0.0, -2e-4]), particles=bodies, contact_rs=1.0,
                  contact_kn=20.0, contact_en=0.5, contact_mu=0.5, quad_h=0.25,
                  name=f"suspension-{box}-{n_bodies}")


def mlp_init(seed: int = 7):
    """Initial weights of the 87-64-64-4 warm-start MLP (parameter order
    W1, b1, W2, b2, W3, b3): Xavier-uniform weights, zero biases."""
    rng = _rng(seed)
    parts = []
    for fan_in, fan_out in ((87, 64), (64, 64), (64, 4)):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-a, a, size=(fan_in, fan_out)).reshape(-1))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


# ------------------------------------------------ Metaball-Imaging inputs
def mi_body(seed: int = 61, n_cp: int = 8, R: float = 10.0):
    """A known metaball (control points about the origin, weights summing to
    R^2) from which a synthetic point hull is sampled."""
    off, k = random_body(_rng(seed), n_cp, R)
    return off - off.mean(0), k


def mi_hull(cp, k, m: int = 2048, dr: float = 0.02):
    """m points on the outer surface of the metaball (cp, k): along m
    Fibonacci directions from the origin, the outermost radius where
    sum k / |x - p|^2 >= 1 (found on a radial grid of step dr, then by 60
    bisections), then translated to their mean (the paper's TOC).  Returns
    the hull [m][3] and the half-spaces of its convex hull [n_pl][4]
    (n . x + d <= 0 inside, scipy.spatial.ConvexHull)."""
    from scipy.spatial import ConvexHull

    cp = np.asarray(cp, dtype=np.float64).reshape(-1, 3)
    k = np.asarray(k, dtype=np.float64)
    i = np.arange(m) + 0.5
    phi = np.arccos(1 - 2 * i / m)
    th = np.pi * (1 + 5 ** 0.5) * i
    dirs = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], axis=1)

    def C(pts):
        d2 = ((pts[..., None, :] - cp) ** 2).sum(-1)
        return (k / d2).sum(-1)

    rmax = float(np.max(np.linalg.norm(cp, axis=1)) + np.sqrt(k.sum())) + 1.0
    r = np.arange(rmax, 0.0, -dr)
    hull = np.zeros((m, 3))
    for j in range(m):
        v = C(dirs[j][None, :] * r[:, None])
        first = int(np.argmax(v >= 1.0))  # outermost sample inside
        lo, hi = r[first], r[first] + dr   # C(lo) >= 1 > C(hi)
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if C(dirs[j] * mid) >= 1.0:
                lo = mid
            else:
                hi = mid
        hull[j] = dirs[j] * lo
    shift = hull.mean(0)
    hull = hull - shift
    planes = ConvexHull(hull).equations.copy()
    return hull, planes, shift


def mi_population(hull, planes, N_I: int, n: int, seed: int = 62, k_scale: float | None = None):
    """Initial GA population [N_I][n][4] (k, x, y, z): control points drawn
    uniformly in the hull's bounding box in batches of 4096, those inside its
    convex hull taken in draw order; weights uniform in (0, 2 k_scale],
    k_scale = (mean hull radius)^2 / n."""
    rng = _rng(seed)
    lo, hi = hull.min(0), hull.max(0)
    if k_scale is None:
        k_scale = float(np.mean(np.linalg.norm(hull, axis=1)) ** 2 / n)
    need = N_I * n
    pts = []
    got = 0
    while got < need:
        c = rng.uniform(lo, hi, size=(4096, 3))
        ok = np.all(c @ planes[:, :3].T + planes[:, 3] <= 0.0, axis=1)
        pts.append(c[ok])
        got += int(ok.sum())
    pop = np.zeros((N_I, n, 4))
    pop[:, :, 1:4] = np.concatenate(pts)[:need].reshape(N_I, n, 3)
    pop[:, :, 0] = np.maximum(rng.uniform(0.0, 2.0 * k_scale, size=(N_I, n)), 1e-3 * k_scale)
    return pop


def mi_draws(E: int, N_I: int, n: int, seed: int = 63):
    """Random numbers of E GA generations: U (uniform [0,1)) and Z (standard
    normal), both [E][N_I][n][4], and the pairings PERM [E][N_I]
    (permutations)."""
    rng = _rng(seed)
    U = rng.random((E, N_I, n, 4))
    Z = rng.standard_normal((E, N_I, n, 4))
    PERM = np.stack([rng.permutation(N_I) for _ in range(E)]).astype(np.int32)
    return U, Z, PERM


# ------------------------------------------------ drafting-kissing-tumbling
def dkt_body(a: float, R: float = 5.0):
    """A body of elongation a: two equal control points at +-a along the body
    x axis, weights summing to R^2 (a = 0: the sphere of radius R).  The set
    C >= 1 is one body while the value at the midpoint, R^2 / a^2, is at
    least 1 (a <= R)."""
    return np.array([[-a, 0.0, 0.0], [a, 0.0, 0.0]]), np.array([0.5 * R * R, 0.5 * R * R])


# Corey shape factors of the paper's designed particles P1-P8 (sec. 4, Table
# T:MP_particles), which the DKT sweep's synthetic bodies are matched to.
DKT_CSF_TARGETS = (1.0, 0.9563, 0.9173, 0.8535, 0.8002, 0.7521, 0.7075, 0.6648)


def dkt_shapes(n_shapes: int = 6, R: float = 5.0, a_max: float = 4.0):
    """Bodies of stepped elongation a = 0 (the sphere of radius R) to a_max
    (dkt_body).  Sizes are made equal in volume by the caller from the
    measured volumes (exact shape scaling p -> s p, k -> s^2 k)."""
    return [dkt_body(a_max * j / max(n_shapes - 1, 1), R) for j in range(n_shapes)]


def dkt_pair(cp, k, D_e: float = 10.0, g: float = 1e-4, tau: float = 0.55) -> Config:
    """Two bodies of one shape settling in a walled box, scaled from the
    paper's set-up (sec. 4): box 0.20 x 0.20 x 0.30 m for a volume-equivalent
    diameter D_e = 0.0125 m, i.e. 16 D_e x 16 D_e x 24 D_e; the bodies start
    0.270 and 0.255 m above the bottom (trailing and leading) with 0.004 m
    between them horizontally; density ratio 2800/976; contact on.  Viscosity
    and gravity (tau 0.55, g 1e-4 at D_e = 10) give the Archimedes number
    (rho_p/rho_f - 1) g D_e^3 / nu^2 = 673, a settling Reynolds number near 20
    (the viscosity printed for this study would put it far below 1, where
    pairs do not tumble)."""
    s = D_e / 0.0125
    nx, ny, nz = int(round(0.20 * s)), int(round(0.20 * s)), int(round(0.30 * s))
    c = np.array([nx / 2, ny / 2])
    bodies = []
    for z, dx in ((0.255, -0.002), (0.270, 0.002)):  # leading first
        bodies.append(Particle(cp_xyz=np.asarray(cp, float), cp_k=np.asarray(k, float),
                               x=np.array([c[0] + dx * s, c[1], z * s]), density=2800.0 / 976.0))
    return Config(nx=nx, ny=ny, nz=nz, periodic=0, tau=tau, rho0=1.0, g_particle=np.array([0.0, 0.0, -g]),
                  bc=BC_IBB, particles=bodies, contact_rs=1.0, contact_kn=20.0, contact_en=0.5, contact_mu=0.5,
                  quad_h=0.25, name=f"dkt-{nx}x{ny}x{nz}")
