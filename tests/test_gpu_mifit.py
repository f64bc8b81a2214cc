"""GPU parity of the Metaball-Imaging fit (paper sec. 2.2; include/mifit.h)
against the FP64 oracle (oracle/mifit.py) on seeded synthetic hulls.

Tolerances (FP64 on both sides; the sums run in different orders):
  fitness F: 1e-12 relative; GA populations after E generations: the same
  individuals in the same order to 1e-12 (selection compares F values that
  differ between individuals far more than the rounding), F to 1e-12;
  gradient search: models and losses to 1e-8 relative after 2 x 60 steps
  (the objective has kinks at f = 1 and f = 2, where a rounding-level
  difference of f changes the slope; over these steps none is crossed
  differently); anomaly cleaning: the same control points zeroed.
"""
import numpy as np
import pytest

import workloads
from oracle import mifit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_10411_amd as m
    m.lib()
    return m


def body(seed, n_cp=8, R=10.0, m=512):
    cp, k = workloads.mi_body(seed=seed, n_cp=n_cp, R=R)
    H, pl, sh = workloads.mi_hull(cp, k, m=m)
    return H, pl, np.concatenate([k[:, None], cp - sh], 1)


@pytest.mark.parametrize("m", [512, 5000])
def test_fitness(mdl, m):
    """One chunk of hull points, and three (the last one ragged) with the
    chunk sums through the workspace."""
    print(f"mifit fitness m={m}", flush=True)
    H, pl, truth = body(70, m=m)
    pop = workloads.mi_population(H, pl, 37, 8, seed=71)
    pop[3] = truth
    Fg = mdl.mi_fitness(H, pop)
    Fo = np.array([mifit.fitness(p, H) for p in pop])
    assert np.abs(Fg - Fo).max() <= 1e-12 * np.abs(Fo).max()
    assert Fg[3] < 1e-20


@pytest.mark.parametrize("N_I,n", [(24, 6), (33, 5)])
def test_ga_generations(mdl, N_I, n):
    """E = 6 generations from the same population and draws (odd N_I: the
    last individual of the pairing is copied)."""
    print(f"mifit GA N_I={N_I} n={n}", flush=True)
    H, pl, _ = body(72, n_cp=5, R=7.0, m=300)
    pop0 = workloads.mi_population(H, pl, N_I, n, seed=73)
    E = 6
    U, Z, PERM = workloads.mi_draws(E, N_I, n, seed=74)
    sx, sk = 0.5, 0.2 * float(pop0[..., 0].mean())
    pg, Fg = mdl.mi_ga(H, pop0, E, 0.6, 0.5, sx, sk, U, Z, PERM)
    po, Fo = mifit.ga(H, pop0, E, 0.6, 0.5, sx, sk, U, Z, PERM)
    assert np.abs(Fg - Fo).max() <= 1e-12 * np.abs(Fo).max()
    assert np.abs(pg - po).max() <= 1e-12 * np.abs(po).max()
    assert np.all(np.diff(Fg) >= 0) and Fg[0] < min(mifit.fitness(p, H) for p in pop0)


def test_gs_batch(mdl):
    """Three models of different hull sizes in one launch (one workgroup
    each): fits and the three losses against the oracle."""
    print("mifit GS batch", flush=True)
    items = [body(75, m=400), body(76, n_cp=8, R=8.0, m=777), body(77, m=1500)]
    rng = np.random.default_rng(78)
    M0 = []
    for H, pl, truth in items:
        M = truth.copy()
        M[:, 1:] += rng.normal(0, 0.5, M[:, 1:].shape)
        M[:, 0] *= rng.uniform(0.7, 1.3, len(M))
        M0.append(M)
    M0 = np.array(M0)
    E, eta = 60, 1e-3
    Mg, Lg = mdl.mi_gs([it[0] for it in items], [it[1] for it in items], M0, E, eta)
    for b, (H, pl, _) in enumerate(items):
        Mo, Lo = mifit.gs(M0[b], H, pl, E, eta)
        print(f"model {b}: L {Lo} max|dM|/|M| {np.abs(Mg[b] - Mo).max() / np.abs(Mo).max():.2e}", flush=True)
        assert np.abs(Mg[b] - Mo).max() <= 1e-8 * np.abs(Mo).max()
        assert np.allclose(Lg[b], Lo, rtol=1e-8, atol=0)
        assert Lg[b][2] < Lg[b][0]


def test_gs_cleans_anomalies(mdl):
    """A start with one negative weight and one control point outside the
    hull: after the first descent both are zeroed, as in the oracle."""
    print("mifit GS cleaning", flush=True)
    H, pl, truth = body(79, n_cp=6, R=8.0, m=600)
    M0 = truth.copy()
    M0[1, 0] = -0.5
    M0[4, 1:] = 3.0 * np.abs(H).max() * np.array([1.0, 0.0, 0.0])
    M0[4, 0] = 0.05
    Mg, Lg = mdl.mi_gs([H], [pl], M0[None], 20, 1e-4)
    Mo, Lo = mifit.gs(M0, H, pl, 20, 1e-4)
    M1 = M0.copy()
    for _ in range(20):
        M1 = M1 - 1e-4 * mifit.gs_grad(M1, H)
    bad = (M1[:, 0] < 0) | ~mifit.inside(M1[:, 1:4], pl)
    assert bad[1] and bad[4]
    assert np.abs(Mg[0] - Mo).max() <= 1e-9 * np.abs(Mo).max()
    assert np.allclose(Lg[0], Lo, rtol=1e-9, atol=0)


def test_fit_pipeline(mdl):
    """Steps 2 and 3 of the method on one synthetic hull: the GA's fittest
    individual starts the gradient search; the fit ends close to the hull
    (the GPU's result is compared with the oracle's)."""
    print("mifit pipeline", flush=True)
    H, pl, truth = body(80, n_cp=6, R=8.0, m=500)
    N_I, n, E = 30, 6, 8
    pop0 = workloads.mi_population(H, pl, N_I, n, seed=81)
    U, Z, PERM = workloads.mi_draws(E, N_I, n, seed=82)
    sx, sk = 0.5, 0.2 * float(pop0[..., 0].mean())
    pg, Fg = mdl.mi_ga(H, pop0, E, 0.6, 0.5, sx, sk, U, Z, PERM)
    po, Fo = mifit.ga(H, pop0, E, 0.6, 0.5, sx, sk, U, Z, PERM)
    assert np.abs(pg[0] - po[0]).max() <= 1e-12 * np.abs(po[0]).max()
    Mg, Lg = mdl.mi_gs([H], [pl], pg[:1], 40, 1e-3)
    Mo, Lo = mifit.gs(po[0], H, pl, 40, 1e-3)
    assert np.abs(Mg[0] - Mo).max() <= 1e-8 * np.abs(Mo).max()
    assert Lg[0][2] < Lg[0][0]
