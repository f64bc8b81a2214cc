"""Pins of the Metaball-Imaging fit oracle (paper sec. 2.2) against
mathematics, not against itself.

- Values: one control point is the ball of radius sqrt(k) (sec. 2.1): on
  its sphere f = 1, so F = 0 and L = 0; at distance r, f = k / r^2.
- The piecewise objective (Eq. GSloss) is continuous at f = 1 and f = 2,
  zero only at f = 1, and its branches are the three written forms.
- The analytic gradient matches central finite differences of the loss.
- The convex-hull test agrees with a cube's and a ball's inside/outside.
- Anomaly cleaning zeroes exactly the negative weights and the control
  points outside the hull.
- Gradient search recovers a known metaball from its own sampled surface:
  the single-point sphere (k and centre, to the O(eta) band that fixed-step
  descent on the |f - 1| branch leaves), an 8-point body to a small
  residual; the loss never increases in the first descent at the paper's
  learning rate.
- GA: mutation changes exactly the genes whose draw is below C_m, by z
  sigma; crossover exchanges whole control points from round(C_c n) on and
  keeps each pair's control points; selection equals a brute-force sort;
  the best fitness never increases (elitism) and a population holding the
  true model returns it.
"""
import numpy as np
import pytest

import workloads
from oracle import mifit


def sphere_hull(k=25.0, m=400, c=(0.0, 0.0, 0.0)):
    i = np.arange(m) + 0.5
    phi = np.arccos(1 - 2 * i / m)
    th = np.pi * (1 + 5 ** 0.5) * i
    d = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    return np.sqrt(k) * d + np.asarray(c)


def test_single_point_is_a_ball():
    k = 25.0
    H = sphere_hull(k)
    M = np.array([[k, 0.0, 0.0, 0.0]])
    f = mifit.values(M, H)
    assert np.abs(f - 1).max() < 1e-14
    assert mifit.fitness(M, H) < 1e-26
    assert mifit.gs_loss(M, H) < 1e-12
    P = np.array([[3.0, 4.0, 12.0]])  # r = 13
    assert mifit.values(M, P)[0] == pytest.approx(k / 169.0, rel=1e-15)


def test_loss_branches_and_continuity():
    eps = 1e-9
    v, _, _ = mifit.loss_terms(np.array([1 - eps, 1.0, 1 + eps, 2 - eps, 2.0, 2 + eps]))
    assert v[0] < 1e-8 and v[1] == 0.0 and v[2] < 1e-8
    assert v[3] == pytest.approx(1.0, abs=1e-8) and v[4] == 1.0 and v[5] == pytest.approx(1.0, abs=1e-8)
    # the written forms in each range
    f = np.array([0.25, 0.5, 1.5, 3.0])
    v, d, _ = mifit.loss_terms(f)
    assert np.allclose(v, [(0.75) ** 2 + 4 - 1, 0.25 + 2 - 1, 0.5, 4.0], rtol=1e-15)
    assert np.allclose(d, [2 * (-0.75) - 16, 2 * (-0.5) - 4, 1.0, 4.0], rtol=1e-15)
    # positive away from the surface, zero on it
    ff = np.linspace(0.05, 5, 400)
    vv, _, _ = mifit.loss_terms(ff)
    assert (vv[np.abs(ff - 1) > 1e-3] > 0).all()


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_finite_differences(seed):
    cp, k = workloads.mi_body(seed=60 + seed, n_cp=5, R=6.0)
    H, pl, sh = workloads.mi_hull(cp, k, m=200)
    rng = np.random.default_rng(seed)
    M = np.concatenate([k[:, None], cp - sh], 1)
    M[:, 1:] += rng.normal(0, 0.4, M[:, 1:].shape)
    M[:, 0] *= rng.uniform(0.6, 1.4, len(k))
    f = mifit.values(M, H)
    # keep clear of the kinks at f = 1 and f = 2 (one-sided slopes differ)
    assert np.min(np.abs(f - 1)) > 1e-4 and np.min(np.abs(f - 2)) > 1e-4
    G = mifit.gs_grad(M, H)
    h = 1e-6
    Gn = np.zeros_like(M)
    for a in range(M.shape[0]):
        for b in range(4):
            Mp, Mm = M.copy(), M.copy()
            Mp[a, b] += h
            Mm[a, b] -= h
            Gn[a, b] = (mifit.gs_loss(Mp, H) - mifit.gs_loss(Mm, H)) / (2 * h)
    assert np.abs(G - Gn).max() < 1e-6 * np.abs(G).max()


def test_convex_hull_test():
    # the unit cube: six planes n . x + d <= 0
    pl = np.array([[1, 0, 0, -1], [-1, 0, 0, 0], [0, 1, 0, -1], [0, -1, 0, 0], [0, 0, 1, -1], [0, 0, -1, 0]], float)
    P = np.array([[0.5, 0.5, 0.5], [1.2, 0.5, 0.5], [0.5, -0.1, 0.5], [0.999, 0.001, 0.5]])
    assert list(mifit.inside(P, pl)) == [True, False, False, True]
    # the hull of points on a sphere of radius 5: inside at 4.5, outside at 5.5
    H = sphere_hull(25.0, 600)
    from scipy.spatial import ConvexHull
    planes = ConvexHull(H).equations
    d = np.random.default_rng(0).normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    assert mifit.inside(4.5 * d, planes).all() and not mifit.inside(5.5 * d, planes).any()


def test_clean_zeroes_the_anomalies():
    pl = np.array([[1, 0, 0, -1], [-1, 0, 0, -1], [0, 1, 0, -1], [0, -1, 0, -1], [0, 0, 1, -1], [0, 0, -1, -1]], float)
    M = np.array([[1.0, 0, 0, 0], [-0.5, 0.1, 0, 0], [2.0, 1.5, 0, 0], [3.0, 0.5, 0.5, -0.9]])
    C = mifit.clean(M, pl)
    assert list(C[:, 0]) == [1.0, 0.0, 0.0, 3.0]
    assert np.array_equal(C[:, 1:], M[:, 1:])


def test_gs_recovers_a_sphere():
    k, c = 25.0, np.array([0.3, -0.2, 0.1])
    H = sphere_hull(k, 300, c)
    from scipy.spatial import ConvexHull
    pl = ConvexHull(H).equations
    M0 = np.array([[0.8 * k, 0.9, 0.4, -0.6]])
    M, L = mifit.gs(M0, H, pl, 1500, 1e-3)
    # the |f - 1| branch has slope 1 on both sides of f = 1 only in sign:
    # fixed-step descent ends in an O(eta) band about the optimum
    assert L[2] < 2e-3 * L[0]
    assert abs(M[0, 0] - k) < 2e-3 * k and np.abs(M[0, 1:] - c).max() < 1e-3
    assert np.abs(mifit.values(M, H) - 1).max() < 2e-3


def test_gs_refines_a_known_body():
    cp, k = workloads.mi_body(seed=61, n_cp=8, R=10.0)
    H, pl, sh = workloads.mi_hull(cp, k, m=512)
    truth = np.concatenate([k[:, None], cp - sh], 1)
    rng = np.random.default_rng(5)
    M0 = truth.copy()
    M0[:, 1:] += rng.normal(0, 0.5, (8, 3))
    M0[:, 0] *= rng.uniform(0.7, 1.3, 8)
    # the loss falls monotonically along the first descent at the paper's rate
    M, Ls = M0.copy(), [mifit.gs_loss(M0, H)]
    for _ in range(200):
        M = M - 1e-3 * mifit.gs_grad(M, H)
        Ls.append(mifit.gs_loss(M, H))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(Ls, Ls[1:]))
    Mg, L = mifit.gs(M0, H, pl, 2000, 1e-3)
    assert L[2] < L[1] < 0.15 * L[0]
    assert np.abs(mifit.values(Mg, H) - 1).max() < 0.04


def test_mutation_and_crossover():
    rng = np.random.default_rng(1)
    pop = rng.uniform(0.5, 1.5, (6, 5, 4))
    U, Z = rng.random((6, 5, 4)), rng.standard_normal((6, 5, 4))
    mut = mifit.mutate(pop, U, Z, 0.6, 0.3, 0.1)
    sig = np.array([0.1, 0.3, 0.3, 0.3])
    changed = U < 0.6
    expect = np.where(changed, pop + Z * sig, pop)
    expect[..., 0] = np.maximum(expect[..., 0], 0)
    assert np.array_equal(mut, expect)
    assert np.array_equal(mut[~changed], pop[~changed])
    perm = np.array([3, 0, 5, 1, 2, 4])
    kids = mifit.crossover(pop, perm, 0.5)  # c = round(2.5) = 3
    for j in range(3):
        a, b = pop[perm[2 * j]], pop[perm[2 * j + 1]]
        assert np.array_equal(kids[2 * j], np.concatenate([a[:3], b[3:]]))
        assert np.array_equal(kids[2 * j + 1], np.concatenate([b[:3], a[3:]]))
        both = np.sort(np.concatenate([kids[2 * j], kids[2 * j + 1]]).view("f8,f8,f8,f8"), axis=0)
        assert np.array_equal(both, np.sort(np.concatenate([a, b]).view("f8,f8,f8,f8"), axis=0))


def test_selection_and_elitism():
    cp, k = workloads.mi_body(seed=64, n_cp=4, R=6.0)
    H, pl, sh = workloads.mi_hull(cp, k, m=150)
    N_I, n, E = 12, 4, 6
    pop0 = workloads.mi_population(H, pl, N_I, n, seed=3)
    assert all(mifit.inside(pop0[a, :, 1:4], pl).all() for a in range(N_I))
    U, Z, PERM = workloads.mi_draws(E, N_I, n, seed=4)
    F0 = sorted(mifit.fitness(m, H) for m in pop0)
    best = [F0[0]]
    pop = pop0
    for e in range(E):
        pop, F = mifit.ga(H, pop, 1, 0.6, 0.5, 0.5, 0.2, U[e:e + 1], Z[e:e + 1], PERM[e:e + 1])
        best.append(F[0])
        # survivors are the N_I smallest of the pool, in order
        assert np.all(np.diff(F) >= 0)
    assert all(b <= a for a, b in zip(best, best[1:]))
    assert best[-1] < best[0]
    # brute-force selection
    pool = np.random.default_rng(2).normal(size=(9, 4, 4))
    Fp = np.array([3.0, 1.0, 2.0, 1.0, 5.0, 0.5, 2.0, 7.0, 1.0])
    s, Fs = mifit.select(pool, Fp, 4)
    assert list(Fs) == [0.5, 1.0, 1.0, 1.0]
    assert np.array_equal(s, pool[[5, 1, 3, 8]])
    # a population holding the true model returns it
    truth = np.concatenate([k[:, None], cp - sh], 1)
    popt = pop0.copy()
    popt[7] = truth
    pt, Ft = mifit.ga(H, popt, 2, 0.6, 0.5, 0.5, 0.2, U[:2], Z[:2], PERM[:2])
    assert Ft[0] <= mifit.fitness(truth, H) + 1e-30 and Ft[0] < 1e-20
