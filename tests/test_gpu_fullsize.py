"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times (the same constructors and default grids;
the ensemble autotuned as the benchmark does): the HIP path against the FP64
oracle over the whole lattice.  Flags, owners and link sets exact; q on every
link; one step from a seeded random state compared at every population of
every fluid node; hydrodynamic forces.

Bounds on one step from deviations d with M = max |d| (a priori, per
population; u32 = 2^-24 the FP32 unit roundoff):
  A post-collision population depends on the 19 pulled inputs with a sum of
  |partial derivatives| K <= |1 - omega| + omega w_i sum_k |1 + 3 e_i . e_k|
  (plus terms of order |u|): at most 11.2, for the rest population at
  tau = 0.6; K = 12 is taken.
  FP32 storage: 250 u32 M.  Input rounding to storage K u32 M; the moments
  (rho - rho0, j) are sums of 19 terms of size <= M, each off by at most
  gamma_18 19 M = 342 u32 M, and enter a population with weights summing to
  at most omega max_i w_i (1 + 3 sum_a |e_ia|) = omega / 3, i.e. 114 omega
  u32 M = 190 u32 M; about ten further roundings of quantities below 4 M add
  40 u32 M; the result is rounded once more.  (The largest measured
  difference is an order of magnitude below.)
  FP16 / BF16 storage: 13 u M + 250 u32 M with u the unit roundoff of the
  stored deviation (2^-11 FP16, 2^-8 BF16): the input state and the result
  are each rounded once to storage.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

AMP = 2e-3


@pytest.fixture(scope="module")
def mdl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_10411_amd as m
    m.lib()
    return m


def same_links(sim, ref):
    ng, dg, og, qg = sim.links()
    no, do, oo, qo = ref.links()
    kg, ko = np.lexsort((dg, ng)), np.lexsort((do, no))
    assert len(ng) == len(no), (len(ng), len(no))
    assert np.array_equal(ng[kg], no[ko]) and np.array_equal(dg[kg], do[ko]) and np.array_equal(og[kg], oo[ko])
    return np.abs(qg[kg] - qo[ko])


def one_step_error(sim, ref, seed):
    """Both sides from the same random state, one step; the largest
    population difference over the fluid nodes and the largest deviation of
    the input."""
    d0 = workloads.random_populations(seed, ref.N, amp=AMP)
    dmax = float(np.abs(d0).max())
    d0 += oracle.feq(1.0, [0, 0, 0])[:, None]  # f0 in place (the arrays are several GB)
    sim.set_populations(d0)
    ref.set_f(d0)
    del d0
    sim.step(1)
    ref.step(1)
    own_g, own_o = sim.owner(), ref.owner()
    assert np.array_equal(own_g, own_o), f"flags differ at {np.flatnonzero(own_g != own_o)[:10]}"
    fl = own_o < 0
    err = 0.0
    fg, fo = sim.populations(), ref.fpost()
    for i in range(19):  # row by row: the full arrays are several GB
        err = max(err, float(np.abs(fg[i, fl] - fo[i, fl]).max()))
    return err, dmax


def forces_match(sim, ref, rel):
    Fg, _ = sim.particle_forces()
    Fo = np.array([ref.particle(p)["F"] for p in range(len(Fg))])
    scale = np.abs(Fo).max()
    assert np.abs(Fg - Fo).max() <= rel * scale, (np.abs(Fg - Fo).max(), scale)


U32 = 2.0 ** -24


def step_bound(storage, dmax):
    b = 250.0 * U32 * dmax
    if storage == workloads.STORE_F16:
        b += 13.0 * 2.0 ** -11 * dmax
    elif storage == workloads.STORE_BF16:
        b += 13.0 * 2.0 ** -8 * dmax
    return b


@pytest.mark.parametrize("storage", [workloads.STORE_F32, workloads.STORE_F16])
def test_settling_128x128x384(mdl, storage):
    """The benchmark workload (one free 8-point body, walls, IBB) at full
    size, FP32 and FP16 storage."""
    cfg = workloads.config2()
    cfg.storage = storage
    print(f"settling 128x128x384 storage {storage}", flush=True)
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    assert np.array_equal(sim.owner(), ref.owner())
    dq = same_links(sim, ref)
    print(f"  links {len(dq)}: median |dq| {np.median(dq):.1e} max {dq.max():.1e}", flush=True)
    assert np.median(dq) < 1e-14 and dq.max() < 2e-7
    err, dmax = one_step_error(sim, ref, seed=31)
    tol = step_bound(storage, dmax)
    print(f"  one step: max |df| {err:.2e} (bound {tol:.1e})", flush=True)
    assert err <= tol
    if storage == workloads.STORE_F32:
        forces_match(sim, ref, 1e-6)
    assert np.array_equal(sim.owner(), ref.owner())
    same_links(sim, ref)
    sim.close()


@pytest.mark.parametrize("storage", [workloads.STORE_F16, workloads.STORE_BF16])
def test_pair_160x160x640(mdl, storage):
    """The two-body drafting workload at full size in its half-precision
    storage forms."""
    cfg = workloads.config3(storage=storage)
    print(f"pair 160x160x640 storage {storage}", flush=True)
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    assert np.array_equal(sim.owner(), ref.owner())
    dq = same_links(sim, ref)
    assert np.median(dq) < 1e-14 and dq.max() < 2e-7
    err, dmax = one_step_error(sim, ref, seed=32)
    tol = step_bound(storage, dmax)
    print(f"  links {len(dq)}; one step: max |df| {err:.2e} (bound {tol:.1e})", flush=True)
    assert err <= tol
    sim.close()


def test_suspension_256_200_bodies(mdl):
    """The 256^3 periodic suspension with 200 bodies and contact at full
    size: flags of all bodies, 1.45 M links, one coupled step; then the warm
    start (an untrained network: the guess is judged by the Newton
    tolerance) finds the plain roots on every link."""
    cfg = workloads.config5(seed=5)
    print("suspension 256^3, 200 bodies", flush=True)
    sim = mdl.Simulation(cfg)
    ref = oracle.Oracle(cfg)
    assert np.array_equal(sim.owner(), ref.owner())
    dq = same_links(sim, ref)
    print(f"  links {len(dq)}: median |dq| {np.median(dq):.1e} p99 {np.quantile(dq, 0.99):.1e} "
          f"max {dq.max():.1e}", flush=True)
    assert np.quantile(dq, 0.99) < 1e-12 and dq.max() < 1e-6
    err, dmax = one_step_error(sim, ref, seed=33)
    tol = step_bound(workloads.STORE_F32, dmax)
    print(f"  one step: max |df| {err:.2e} (bound {tol:.1e})", flush=True)
    assert err <= tol
    forces_match(sim, ref, 1e-6)
    # after the step q follows the moved poses, which differ by the FP32
    # rounding of the fluid's forces (the bound of the moving-body tests)
    dq = same_links(sim, ref)
    print(f"  links after the step: median |dq| {np.median(dq):.1e} max {dq.max():.1e}", flush=True)
    assert np.median(dq) < 1e-7 and dq.max() < 1e-4
    del ref
    sim.close()
    # warm start against plain, one step from the initial state
    warm = mdl.Simulation(cfg)
    warm.set_warmstart(mdl.Mlp(workloads.mlp_init(5)))
    plain = mdl.Simulation(cfg)
    warm.step(1)
    plain.step(1)
    nw, dw, ow, qw = warm.links()
    npl, dp, op, qp = plain.links()
    kw, kp = np.lexsort((dw, nw)), np.lexsort((dp, npl))
    assert np.array_equal(nw[kw], npl[kp]) and np.array_equal(dw[kw], dp[kp]) and np.array_equal(ow[kw], op[kp])
    dq = np.abs(qw[kw] - qp[kp])
    print(f"  warm vs plain: {len(dq)} links, max |dq| {dq.max():.1e}", flush=True)
    assert dq.max() < 1e-12
    warm.close()
    plain.close()


def test_ensemble_64_cases(mdl):
    """The 64-case settling ensemble (87 M nodes), autotuned as the
    benchmark runs it, two steps; four cases (smallest, largest and two
    others) against the oracle at every fluid population."""
    cfgs = workloads.config4()
    print("ensemble of 64 settling cases", flush=True)
    ens = mdl.Ensemble(cfgs)
    tiles, bw = ens.autotune(budget_ms=1000.0)
    print(f"  tiles {sorted(set(tiles))}, waves per block {bw}", flush=True)
    ens.step(2)
    ens.sync()
    sizes = [c.nx * c.ny * c.nz for c in cfgs]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 42})
    for b in pick:
        ref = oracle.Oracle(cfgs[b])
        ref.step(2)
        sim = ens.cases[b]
        own_g, own_o = sim.owner(), ref.owner()
        assert np.array_equal(own_g, own_o), f"case {b}: flags differ"
        same_links(sim, ref)
        fl = own_o < 0
        fg, fo = sim.populations(), ref.fpost()
        w = oracle.feq(1.0, [0, 0, 0])
        err = max(float(np.abs(fg[i, fl] - fo[i, fl]).max()) for i in range(19))
        dmax = max(float(np.abs(fo[i, fl] - w[i]).max()) for i in range(19))
        tol = 2 * step_bound(workloads.STORE_F32, dmax)  # two steps
        print(f"  case {b} ({cfgs[b].nx}x{cfgs[b].ny}x{cfgs[b].nz}): max |df| {err:.2e} (bound {tol:.1e})",
              flush=True)
        assert err <= tol
    ens.close()
