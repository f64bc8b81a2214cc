"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Tolerances (FP32 storage of deviations f - w rho0, FP32 collision, FP64
geometry, forces and rigid body):
  flags, owners, link sets: exact;  q: 1e-12 on well-conditioned links;
  max |du|/U <= 1e-5 and max |drho| <= 1e-7 over fluid nodes (U = max |u| of
  the oracle); hydrodynamic force |dF|/|F| <= 1e-4; particle |dx| <= 1e-4 lu.
The FP32 bound follows from the storage: deviations of size d carry a
relative rounding of 6e-8 per step, accumulated over the compared steps.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_10411_amd as m
    m.lib()
    return m


def compare_fields(sim, ref, du_tol=1e-5, drho_tol=1e-7, label=""):
    own_g, own_o = sim.owner(), ref.owner()
    assert np.array_equal(own_g, own_o), f"{label}: flags differ at {np.flatnonzero(own_g != own_o)[:10]}"
    fl = own_o < 0
    rho_g, u_g = sim.macros()
    rho_o, u_o = ref.macros()
    U = np.abs(u_o[fl]).max()
    du = np.abs(u_g[fl] - u_o[fl]).max() / U
    drho = np.abs(rho_g[fl] - rho_o[fl]).max()
    print(f"{label}: U={U:.3e} max|du|/U={du:.3e} max|drho|={drho:.3e}", flush=True)
    assert du <= du_tol, f"{label}: max|du|/U = {du}"
    assert drho <= drho_tol, f"{label}: max|drho| = {drho}"
    return du, drho


# Cases with fast bodies (contact tests: U ~ 0.05-0.08, ten to a hundred
# times the settling cases) carry density deviations ~ 3 U^2 ~ 1e-2, whose
# FP32 storage rounding (6e-8 relative per step) shows in rho at the 1e-7
# level after tens of steps: their density bound is 1e-6 (velocity 1e-5).
DRHO_FAST = 1e-6


def compare_torque(Tg, po, R, label=""):
    """Momentum-exchange torque about the centroid against the oracle's, to
    1e-4 of the larger of |T| and a lever arm (the body radius) times 1e-2
    |F| (a symmetric body's torque is zero up to rounding)."""
    To, Fo = po["T"], po["F"]
    scale = max(np.abs(To).max(), 1e-2 * R * np.abs(Fo).max())
    err = np.abs(np.asarray(Tg) - To).max() / scale
    print(f"{label}: |T|={np.abs(To).max():.3e} max|dT|/scale={err:.2e}", flush=True)
    assert err <= 1e-4, f"{label}: torque {Tg} vs {To}"


def compare_links(sim, ref):
    ng, dg, og, qg = sim.links()
    no, do, oo, qo = ref.links()
    kg = np.lexsort((dg, ng))
    ko = np.lexsort((do, no))
    assert np.array_equal(ng[kg], no[ko]) and np.array_equal(dg[kg], do[ko])
    assert np.array_equal(og[kg], oo[ko])
    dq = np.abs(qg[kg] - qo[ko])
    return dq


@pytest.mark.parametrize("center", ["integer", "half"])
def test_flags_links_q_sphere(mdl, center):
    cfg = workloads.config1(center=center)
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    own = sim.owner()
    assert np.array_equal(own, ref.owner())
    assert (own >= 0).sum() == (2109 if center == "integer" else 2176)
    dq = compare_links(sim, ref)
    assert len(dq) == (4530 if center == "integer" else 4704)
    assert np.median(dq) < 1e-14 and dq.max() < 2e-7
    ns, nl = sim.metaball_flag()
    assert ns == (own >= 0).sum() and nl == len(dq)


@pytest.mark.parametrize("seed", [1, 2])
def test_flags_links_q_random_body(mdl, seed):
    off, k = workloads.random_body(np.random.Generator(np.random.PCG64(seed)), 12, 7.0)
    cfg = workloads.Config(nx=48, ny=40, nz=44, periodic=7, tau=0.8, bc=workloads.BC_IBB,
                           particles=[workloads.Particle(cp_xyz=off, cp_k=k,
                                                         x=np.array([47.3, 19.6, 1.1]),
                                                         density=1.0, mode=workloads.MODE_KINEMATIC)])
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    assert np.array_equal(sim.owner(), ref.owner())
    dq = compare_links(sim, ref)
    assert np.quantile(dq, 0.99) < 1e-12 and dq.max() < 1e-6


@pytest.mark.parametrize("case", ["six_periodic", "forty"])
def test_flags_links_q_many_bodies(mdl, case):
    """Many bodies at their initial poses (the same on both sides): flags, the
    body-major link list and every link fraction against the oracle.  The
    solver stages one body's control points per wave at a time, so a wave
    whose eight links span two bodies takes a turn per body; the lists here
    hold such waves at most body boundaries."""
    if case == "six_periodic":
        cfg = workloads.suspension_small()
    else:
        cfg = workloads.suspension_small(n_bodies=40, box=64, seed=52)
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    assert np.array_equal(sim.owner(), ref.owner())
    dq = compare_links(sim, ref)
    _, _, og, _ = sim.links()  # list order: eight consecutive links per wave of the solver
    spans = sum(1 for w in range(0, len(og), 8) if len(set(og[w:w + 8].tolist())) > 1)
    print(f"{case}: {len(og)} links, {spans} waves across a body boundary, max |dq| {dq.max():.1e}", flush=True)
    assert spans >= 3
    assert np.quantile(dq, 0.99) < 1e-12 and dq.max() < 1e-6


@pytest.mark.parametrize("bc", [workloads.BC_SBB, workloads.BC_IBB])
def test_config1_200_steps(mdl, bc):
    """64^3 periodic, fixed sphere k = 64, body force 1e-6, 200 steps;
    fields at steps 1, 10, 200 and the force."""
    cfg = workloads.config1(bc=bc)
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    done = 0
    for upto in (1, 10, 200):
        sim.step(upto - done)
        ref.step(upto - done)
        done = upto
        compare_fields(sim, ref, label=f"cfg1 bc={bc} step {upto}")
        Fg, Tg = sim.particle_forces()
        po = ref.particle(0)
        Fo = po["F"]
        assert np.abs(Fg[0] - Fo).max() <= 1e-4 * np.abs(Fo).max()
        compare_torque(Tg[0], po, 8.0, label=f"cfg1 bc={bc} step {upto} torque")


@pytest.mark.parametrize("bc", [workloads.BC_SBB, workloads.BC_IBB])
def test_settling_body_with_refill(mdl, bc):
    """Free body falling fast enough to cover and uncover nodes every few
    steps: flags, fields, forces and trajectory against the oracle."""
    cfg = workloads.small_settling(n=32, nz=56, R=5.0, g=5e-4, bc=bc)
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    refilled = 0
    for k in range(6):
        sim.step(10)
        for _ in range(10):
            ref.step(1)
            refilled += ref.n_refilled
        compare_fields(sim, ref, label=f"settle bc={bc} step {10 * (k + 1)}")
        # same links; q follows the pose, which differs from the oracle's by
        # ~1e-7 (FP32 fluid), more on grazing links
        dq = compare_links(sim, ref)
        assert np.median(dq) < 1e-7 and dq.max() < 1e-4
        pg, po = sim.particles()[0], ref.particle(0)
        assert np.abs(pg["x"] - po["x"]).max() < 1e-6
        assert np.abs(pg["v"] - po["v"]).max() < 1e-6 * max(1.0, np.abs(po["v"]).max())
        assert np.abs(pg["F"] - po["F"]).max() <= 1e-4 * np.abs(po["F"]).max()
        compare_torque(pg["T"], po, 5.0, label=f"settle bc={bc} step {10 * (k + 1)} torque")
        assert np.abs(pg["omega"] - po["omega"]).max() <= 1e-6 * max(np.abs(po["omega"]).max(), 1e-3)
    assert refilled > 0


def test_two_bodies(mdl):
    cfg = workloads.two_body()
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    sim.step(40)
    ref.step(40)
    compare_fields(sim, ref, label="two bodies step 40")
    for j in range(2):
        assert np.abs(sim.particles()[j]["x"] - ref.particle(j)["x"]).max() < 1e-6


def test_one_step_from_random_state(mdl):
    """A random post-stream state (not an equilibrium) streamed, bounced and
    collided once, periodic and walled, every population compared."""
    for cfg in (workloads.config1(bc=workloads.BC_IBB, n=32), workloads.small_settling(n=24, nz=32, R=4.0)):
        N = cfg.nx * cfg.ny * cfg.nz
        f0 = oracle.feq(1.0, [0, 0, 0])[:, None] + workloads.random_populations(3, N, amp=2e-3)
        sim = mdl.Simulation(cfg)
        ref = oracle.Oracle(cfg)
        sim.set_populations(f0)
        ref.set_f(f0)
        sim.step(1)
        ref.step(1)
        fl = ref.owner() < 0
        fg = sim.populations()
        fo = ref.fpost()
        err = np.abs(fg[:, fl] - fo[:, fl]).max()
        print(f"one step {cfg.name}: max|df| = {err:.2e}", flush=True)
        assert err < 2e-9


def _half_step_bound(storage, dmax):
    """A priori bound on one step from deviations of size <= dmax with 16-bit
    storage (derivation in test_gpu_fullsize.py): the input and the result
    each rounded once to storage, the collision's sensitivity to its inputs
    at most 12, plus the FP32 arithmetic."""
    u = 2.0 ** -11 if storage == workloads.STORE_F16 else 2.0 ** -8
    return 13.0 * u * dmax + 250.0 * 2.0 ** -24 * dmax


def _box(nx, ny, nz, periodic, storage, g=(0.0, 0.0, 0.0)):
    return workloads.Config(nx=nx, ny=ny, nz=nz, periodic=periodic, tau=0.6, storage=storage,
                            g_fluid=np.array(g))


@pytest.mark.parametrize("storage", [workloads.STORE_F16, workloads.STORE_BF16])
@pytest.mark.parametrize("case", ["periodic-32", "periodic-200", "walls-136", "walls-odd-37", "body-24",
                                  "periodic-4", "walls-4", "periodic-256"])
def test_one_step_half_storage_node_pairs(mdl, storage, case):
    """16-bit storage streams node pairs with 32-bit accesses when nx is even:
    a wave per 128 x of a row when nx is a multiple of 128, else 64 pairs in
    lattice order with rows wrapping inside the wave (shifts across lanes,
    extra loads at row and wave ends, periodic wrap and walls along x, idle
    lanes past the end); odd nx takes the one-node form.  One step from a random state, every population
    of every fluid node against the oracle within the rounding bound."""
    if case == "periodic-32":
        cfg = _box(32, 10, 12, 7, storage, g=(1e-5, -2e-5, 3e-5))
    elif case == "periodic-200":
        cfg = _box(200, 6, 8, 7, storage, g=(2e-5, 0.0, -1e-5))
    elif case == "walls-136":
        cfg = _box(136, 7, 9, 0, storage)
    elif case == "walls-odd-37":
        cfg = _box(37, 9, 8, 2, storage)
    elif case == "periodic-4":  # the narrowest even row (sizes start at 3): two pairs
        cfg = _box(4, 6, 5, 7, storage, g=(1e-5, 1e-5, 0.0))
    elif case == "walls-4":
        cfg = _box(4, 5, 6, 6, storage)
    elif case == "periodic-256":  # nx a multiple of 128: a wave per 128 x of a row
        cfg = _box(256, 4, 5, 7, storage, g=(-1e-5, 2e-5, 1e-5))
    else:
        cfg = workloads.small_settling(n=24, nz=32, R=4.0)
        cfg.storage = storage
    print(f"half storage one step: {case} storage {storage}", flush=True)
    N = cfg.nx * cfg.ny * cfg.nz
    d0 = workloads.random_populations(5, N, amp=2e-3)
    f0 = oracle.feq(1.0, [0, 0, 0])[:, None] + d0
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    sim.set_populations(f0)
    ref.set_f(f0)
    sim.step(1)
    ref.step(1)
    fl = ref.owner() < 0
    assert np.array_equal(sim.owner(), ref.owner())
    err = np.abs(sim.populations()[:, fl] - ref.fpost()[:, fl]).max()
    tol = _half_step_bound(storage, np.abs(d0).max())
    print(f"  max|df| = {err:.2e} (bound {tol:.1e})", flush=True)
    assert err <= tol
    sim.close()


def test_comoving_equilibrium_on_gpu(mdl):
    U = np.array([0.02, 0.011, -0.007])
    cfg = workloads.comoving(U=U, n=24)
    sim = mdl.Simulation(cfg)
    N = cfg.nx * cfg.ny * cfg.nz
    feq = oracle.feq(1.0, U)
    sim.set_populations(np.tile(feq[:, None], (1, N)), post_collision=True)
    sim.step(60)
    fl = sim.owner() < 0
    f = sim.populations()
    assert np.abs(f[:, fl] - feq[:, None]).max() < 2e-8
    # the oracle gives F = 0 to 1e-13; FP32 populations leave a residue of
    # FP32 rounding summed over ~1e3 links, against a drag scale
    # 6 pi mu R |U| ~ 0.1 for this body
    assert np.abs(sim.particle_forces()[0]).max() < 5e-6


def test_poiseuille_on_gpu(mdl):
    tau = 0.5 + np.sqrt(3) / 4
    H, g = 32, 1e-6
    cfg = workloads.poiseuille(tau, H=H, g=g)
    sim = mdl.Simulation(cfg)
    sim.step(30000, coupled=False)
    rho, u = sim.macros()
    nu = (tau - 0.5) / 3
    eta = np.arange(H) - (H - 1) / 2
    ua = g / (2 * nu) * ((H / 2) ** 2 - eta ** 2)
    ux = u[:, 0].reshape(cfg.nz, cfg.ny, cfg.nx)
    err = np.abs(ux - ua[None, :, None]).max() / ua.max()
    print(f"poiseuille FP32: rel err {err:.2e}", flush=True)
    # FP32 steady state: each step rounds the stored deviations to 2^-24
    # relative, and the iteration contracts the slowest mode by only
    # pi^2 nu / H^2 ~ 1/720 per step, so its fixed point sits ~720 x 6e-8
    # ~ 4e-5 of the deviations away from the exact one; the profile's
    # relative error is a few times that
    assert err < 2e-4


def test_fluid_only_then_flag_and_refill(mdl):
    """LBM_STEP_FLUID_ONLY keeps geometry; an external move followed by
    metaball_flag and refill matches the oracle's flags and refill count."""
    cfg = workloads.small_settling(n=28, nz=40, R=4.0)
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    sim.step(5, coupled=False)
    own0 = sim.owner()
    assert np.array_equal(own0, ref.owner())
    st = sim.particles()
    st[0]["x"] = st[0]["x"] + np.array([0.6, -0.4, -0.9])
    sim.set_particles(st)
    ns, nl = sim.metaball_flag()
    p = ref.particle(0)
    ref.set_particle_state(0, st[0]["x"], st[0]["quat"], p["v"], p["omega"])
    ref.reflag()
    own1 = sim.owner()
    assert np.array_equal(own1, ref.owner())
    assert nl == ref.n_links and ns == (own1 >= 0).sum()
    n_ref = sim.refill()
    assert n_ref == int(((own0 >= 0) & (own1 < 0)).sum()) and n_ref > 0


@pytest.mark.parametrize("move", [(0.6, -0.4, -0.9), (2.6, -1.7, 3.2), (-4.0, 3.0, -12.25)])
def test_moved_body_keeps_matching_flags_links_and_fields(mdl, move):
    """A settling body moved from outside (set_particles, metaball_flag,
    refill) by about a node, by several nodes and by more than its size, then
    stepped on from the oracle's state (the oracle's re-flag refills nothing,
    so both continue from its populations): the flags of every later step,
    the links and the fields match the oracle's -- the region work follows
    the moved body and nothing of the old pose is left behind."""
    cfg = workloads.small_settling(n=32, nz=56, R=5.0, g=5e-4)
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    sim.step(8)
    ref.step(8)
    assert np.array_equal(sim.owner(), ref.owner())
    st = sim.particles()
    p = ref.particle(0)
    st[0]["x"] = p["x"] + np.array(move)
    st[0]["v"], st[0]["omega"], st[0]["quat"] = p["v"], p["omega"], p["quat"]
    sim.set_particles(st)
    sim.metaball_flag()
    own0 = ref.owner()
    ref.set_particle_state(0, st[0]["x"], p["quat"], p["v"], p["omega"])
    ref.reflag()
    own1 = sim.owner()
    assert np.array_equal(own1, ref.owner())
    assert sim.refill() == int(((own0 >= 0) & (own1 < 0)).sum())
    sim.set_populations(ref.f(), post_collision=False)
    for k in range(4):
        sim.step(3)
        ref.step(3)
        compare_fields(sim, ref, label=f"{3 * (k + 1)} steps after a move by {move}")
    dq = compare_links(sim, ref)
    assert np.median(dq) < 1e-7 and dq.max() < 1e-4
    assert np.abs(sim.particles()[0]["x"] - ref.particle(0)["x"]).max() < 1e-6


def test_run_twice_bitwise_identical(mdl):
    cfg = workloads.small_settling(n=24, nz=40, R=4.0, g=5e-4)
    out = []
    for _ in range(2):
        sim = mdl.Simulation(cfg)
        sim.step(30)
        out.append((sim.populations(), sim.particles()[0]["x"], sim.particle_forces()[0]))
        sim.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])


@pytest.mark.parametrize("storage,tol", [(workloads.STORE_F16, 5e-3), (workloads.STORE_BF16, 5e-2)])
def test_half_storage_error_vs_oracle(mdl, storage, tol):
    """FP16 / BF16 storage of deviations with FP32 collision: the error
    against the FP64 oracle is reported; bounded loosely here."""
    cfg = workloads.small_settling(n=32, nz=56, R=5.0, g=5e-4)
    cfg.storage = storage
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    sim.step(40)
    ref.step(40)
    fl = ref.owner() < 0
    rho_g, u_g = sim.macros()
    rho_o, u_o = ref.macros()
    U = np.abs(u_o[fl]).max()
    du = np.abs(u_g[fl] - u_o[fl]).max() / U
    dx = np.abs(sim.particles()[0]["x"] - ref.particle(0)["x"]).max()
    print(f"storage {storage}: max|du|/U = {du:.2e}, |dx| = {dx:.2e}", flush=True)
    assert du < tol and dx < 1e-3


def _compare_particles(sim, ref, cfg, tol_x, tol_v):
    L = np.array([cfg.nx, cfg.ny, cfg.nz], float)
    per = np.array([(cfg.periodic >> a) & 1 for a in range(3)], bool)
    gs = sim.particles()
    for j in range(len(cfg.particles)):
        po = ref.particle(j)
        dx = gs[j]["x"] - po["x"]
        dx[per] -= L[per] * np.round(dx[per] / L[per])  # the library keeps periodic centroids in the box
        assert np.abs(dx).max() < tol_x, (j, dx)
        assert np.abs(gs[j]["v"] - po["v"]).max() < tol_v, (j, gs[j]["v"], po["v"])
        assert np.abs(gs[j]["omega"] - po["omega"]).max() < tol_v
    return max(np.abs(gs[j]["x"] - ref.particle(j)["x"]).max() for j in range(len(cfg.particles)))


def test_contact_pair_collision(mdl):
    """Two dense spheres driven into each other: sphero-metaball contact
    (stationary point, Taylor projection, spring-dashpot with friction) on
    the GPU against the oracle, through the collision and rebound."""
    cfg = workloads.contact_pair()
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    for k in range(6):
        sim.step(10)
        ref.step(10)
        compare_fields(sim, ref, drho_tol=DRHO_FAST, label=f"contact pair step {10 * (k + 1)}")
        _compare_particles(sim, ref, cfg, 1e-5, 1e-5)
    nc, nf = sim.contact_stats()
    assert nc == ref.n_contacts and nc > 0 and nf == 0


def test_body_lands_on_floor(mdl):
    cfg = workloads.settle_on_floor()
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    for k in range(5):
        sim.step(40)
        ref.step(40)
        compare_fields(sim, ref, drho_tol=DRHO_FAST, label=f"floor step {40 * (k + 1)}")
        _compare_particles(sim, ref, cfg, 1e-5, 1e-5)
    nc, nf = sim.contact_stats()
    assert nc > 0 and nf == 0
    assert abs(nc - ref.n_contacts) <= 2


def test_periodic_suspension_small(mdl):
    """Six bodies in a periodic box with the fluid counter-force: multi-body
    flags (lowest index owns shared nodes), links, refills and minimum-image
    geometry across the periodic faces."""
    cfg = workloads.suspension_small()
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    assert np.allclose(sim.g_fluid(), ref.g_fluid, rtol=1e-12, atol=1e-18)
    for k in range(3):
        sim.step(20)
        ref.step(20)
        compare_fields(sim, ref, drho_tol=DRHO_FAST, label=f"suspension step {20 * (k + 1)}")
        dq = compare_links(sim, ref)
        # q follows the poses, which differ by up to the 1e-6 position bound
        # for these fast bodies (velocities up to 0.05)
        assert np.median(dq) < 1e-6 and dq.max() < 1e-4
        _compare_particles(sim, ref, cfg, 1e-6, 1e-7)


def test_periodic_suspension_many_bodies(mdl):
    """Forty bodies with contact (more than the one-block rigid-body kernel
    holds in LDS: contacts of all pairs and faces over many blocks, then one
    thread per body) against the oracle: fields, links, particles, contact
    counts."""
    cfg = workloads.suspension_small(n_bodies=40, box=64, seed=52)
    assert len(cfg.particles) == 40
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    for k in range(2):
        sim.step(15)
        ref.step(15)
        compare_fields(sim, ref, label=f"40-body suspension step {15 * (k + 1)}")
        dq = compare_links(sim, ref)
        assert np.median(dq) < 1e-7 and dq.max() < 1e-4
        _compare_particles(sim, ref, cfg, 1e-6, 1e-7)
        gs = sim.particles()
        for j in range(len(cfg.particles)):
            po = ref.particle(j)
            compare_torque(gs[j]["T"], po, 5.0, label=f"40-body step {15 * (k + 1)} body {j} torque")
    nc, nf = sim.contact_stats()
    assert nc == ref.n_contacts and nf == 0
    print(f"40-body suspension: {nc} contacts", flush=True)


_TR_STEPS = (50, 100, 200, 400)


@pytest.fixture(scope="module")
def drafting_oracle():
    """FP64 oracle snapshots of the two-body drafting case at 0.4 scale
    (64 x 64 x 256, bodies of 6 and 12 control points, gravity raised to
    2e-4 so that they move within the compared steps)."""
    cfg = workloads.config3(scale=0.4, storage=workloads.STORE_F32)
    cfg.g_particle = np.array([0.0, 0.0, -2e-4])
    ref = oracle.Oracle(cfg)
    snaps, done = {}, 0
    for s in _TR_STEPS:
        ref.step(s - done)
        done = s
        rho, u = ref.macros()
        snaps[s] = (ref.owner() < 0, u, [ref.particle(j)["x"].copy() for j in range(2)])
    return cfg, snaps


@pytest.mark.parametrize("storage,tol_u,tol_x", [(workloads.STORE_F32, 1e-5, 1e-5), (workloads.STORE_F16, 5e-3, 2e-3),
                                                 (workloads.STORE_BF16, 5e-2, 2e-2)])
def test_storage_error_time_resolved(mdl, drafting_oracle, storage, tol_u, tol_x):
    """Error of each storage type against the FP64 oracle along the
    trajectory (max |du|/U over fluid nodes, particle |dx|), printed per
    checkpoint."""
    cfg0, snaps = drafting_oracle
    cfg = cfg0.copy()
    cfg.storage = storage
    sim = mdl.Simulation(cfg)
    done = 0
    for s in _TR_STEPS:
        sim.step(s - done)
        done = s
        fl, u_o, xs = snaps[s]
        _, u_g = sim.macros()
        fl = fl & (sim.owner() < 0)
        U = np.abs(u_o[fl]).max()
        du = np.abs(u_g[fl] - u_o[fl]).max() / U
        dx = max(np.abs(p["x"] - x).max() for p, x in zip(sim.particles(), xs))
        print(f"storage {storage} step {s}: U={U:.3e} max|du|/U={du:.2e} |dx|={dx:.2e}", flush=True)
        assert du < tol_u and dx < tol_x
    sim.close()


def test_contact_pair_paper_subcycling(mdl):
    """The paper's DEM sub-cycling, 100 rigid-body sub-steps per lattice
    step (DEM step 2e-6 s against the LBM step 2e-4 s): the head-on pair with
    contact against the oracle through the collision (loads held over the
    sub-steps, contacts recomputed at each)."""
    cfg = workloads.contact_pair()
    cfg.n_sub = 100
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    for k in range(4):
        sim.step(10)
        ref.step(10)
        compare_fields(sim, ref, drho_tol=DRHO_FAST, label=f"contact pair n_sub=100 step {10 * (k + 1)}")
        _compare_particles(sim, ref, cfg, 1e-5, 1e-5)
    nc, nf = sim.contact_stats()
    assert nc == ref.n_contacts and nc > 100 and nf == 0
    print(f"n_sub = 100: {nc} contacts over {40 * 100} sub-steps", flush=True)


def test_sphero_metaball_link_level(mdl):
    """Link fractions on the sphero-metaball surface (sec. 2.3.2, q from
    f = c_0 with c_0 depending on R_s; the inner body at c_0 = s^2, R_s = 1):
    the same link set, q against the oracle, then 30 coupled steps of a
    settling body with covering and refilling."""
    cfg = workloads.small_settling(n=32, nz=56, R=5.0, g=5e-4)
    cfg.contact_rs, cfg.link_c0 = 1.0, 1
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    dq = compare_links(sim, ref)
    print(f"c_0 links: |dq| p99 {np.quantile(dq, 0.99):.2e} max {dq.max():.2e}", flush=True)
    assert np.quantile(dq, 0.99) < 1e-12 and dq.max() < 2e-7
    q1 = ref.links()[3]
    assert (q1 >= 1.0).sum() > 0 and (q1 < 1e-9).sum() > 0  # both fallbacks occur
    for k in range(3):
        sim.step(10)
        ref.step(10)
        compare_fields(sim, ref, label=f"c_0 settle step {10 * (k + 1)}")
        dq = compare_links(sim, ref)
        assert np.median(dq) < 1e-7 and dq.max() < 1e-4
        assert np.abs(sim.particles()[0]["x"] - ref.particle(0)["x"]).max() < 1e-6


def test_kernel_timing_every_nth_step(mdl):
    """lbm_timing_enable's stride: with every = 4, ten of forty steps have
    their stream-collide timed; with 1 every step; with timing off none."""
    cfg = workloads.small_settling()
    sim = mdl.Simulation(cfg)
    sim.timing(True, every=4)
    sim.timing_read()
    sim.step(40)
    ms, n, nodes = sim.timing_read()
    assert n == 10 and ms > 0.0 and 0 < nodes <= cfg.n_nodes
    sim.timing(True)
    sim.step(6)
    assert sim.timing_read()[1] == 6
    sim.timing(False)
    sim.step(3)
    assert sim.timing_read()[1] == 0
    sim.close()
