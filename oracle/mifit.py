"""FP64 oracle of the Metaball-Imaging fit (paper sec. 2.2): the genetic
algorithm that captures a particle's principal outer contour and the gradient
search that refines it.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the tests and the
benchmark's baseline may use it; the product library never does.

A metaball model M holds n control points, each (k, x, y, z) with k > 0;
M is an array [n][4] in that order (the genes of one individual, four per
control point).  Its value at a point h is f(h; M) = sum_j k_j / |h - p_j|^2
(sec. 2.1, Eq. metaballM); f = 1 on the surface.  The input is the point hull
H [m][3] of one particle, already centred at the origin (the paper's TOC), and
the half-spaces of its convex hull, planes [n_pl][4] with n . p + d <= 0
inside (the paper's point-in-hull linear program decides whether p is a
convex combination of the hull points, which is exactly this test).

Functions, in the paper's order:
  values        f at every hull point (sec. 2.2, Evaluation: f^l_{H_i}(M))
  fitness       F(M) = sum_i (f_i - 1)^2 (sec. 2.2, Evaluation)
  gs_loss       the piecewise objective of Eq. GSloss
  gs_grad       its gradient with respect to every gene (chain rule of the
                definitions above)
  clean         anomaly detection: control points outside H and negative
                weights get weight zero (sec. 2.2, Anomaly Detection)
  gs            Alg. GS: E gradient-descent steps, cleaning, E more steps
  mutate, crossover, select, ga
                Alg. GA: per generation mutation, crossover, evaluation and
                selection of the N_I fittest

Readings of points the paper leaves open (also listed in the design notes):
  - Eq. GSloss covers f >= 0; with a negative weight f can be negative: the
    f < 1 branch is used there with 1/f taken as 1/max(f, EPS_F) (no
    gradient from that term below EPS_F).  At f = 1 the |f - 1| branch has
    slope +1 (f >= 1) and the f < 1 branch slope -1; at f = 2 the branches
    meet with slopes 1 and 2.  The loss is the sum over hull points as
    written; the learning rate absorbs the hull size.
  - Mutation: each gene changes with probability C_m by a normal step of
    standard deviation sigma_k (weights) or sigma_x (coordinates); a weight
    that would fall below zero is set to zero (weights are positive by
    definition of the metaball).
  - Crossover: the population is paired by a random permutation (pairs
    (perm[2j], perm[2j+1])); the crossover point is c = round(C_c * n) whole
    control points; the two children swap their control points from c on.
  - Selection: from the pool of parents, mutants and children (3 N_I
    individuals, in that order) the N_I of smallest F survive, ties to the
    lower pool index (elitist: the best F never increases).
  - The initial population (control points inside H, positive weights) and
    every random number are inputs.
"""
from __future__ import annotations

import numpy as np

EPS_F = 1e-12   # floor of f in the 1/f term of the loss


# ----------------------------------------------------------- evaluation
def values(M, H):
    """f(H_i; M) for every hull point: sum_j k_j / |H_i - p_j|^2."""
    M = np.asarray(M, dtype=np.float64).reshape(-1, 4)
    H = np.asarray(H, dtype=np.float64).reshape(-1, 3)
    d = H[:, None, :] - M[None, :, 1:4]          # [m][n][3]
    r2 = (d * d).sum(-1)                          # [m][n]
    return (M[None, :, 0] / r2).sum(1)


def fitness(M, H):
    """F(M) = sum_i (f_i - 1)^2 (the GA's fitness score; smaller is fitter)."""
    f = values(M, H)
    return float(((f - 1.0) ** 2).sum())


# ----------------------------------------------------------- gradient search
def loss_terms(f):
    """The per-point terms of Eq. GSloss and their derivatives d/df."""
    f = np.asarray(f, dtype=np.float64)
    fc = np.maximum(f, EPS_F)
    hi = f >= 2.0
    mid = (f >= 1.0) & ~hi
    lo = f < 1.0
    val = np.where(hi, (f - 1.0) ** 2, np.where(mid, np.abs(f - 1.0), (f - 1.0) ** 2 + 1.0 / fc - 1.0))
    der = np.where(hi, 2.0 * (f - 1.0), np.where(mid, 1.0,
                   2.0 * (f - 1.0) - np.where(f > EPS_F, 1.0 / (fc * fc), 0.0)))
    return val, der, lo


def gs_loss(M, H):
    """L(M) of Eq. GSloss, summed over the hull points."""
    v, _, _ = loss_terms(values(M, H))
    return float(v.sum())


def gs_grad(M, H):
    """dL/dM [n][4]: dL/dk_j = sum_i l'(f_i) / r_ij^2,
    dL/dp_j = sum_i l'(f_i) 2 k_j (H_i - p_j) / r_ij^4."""
    M = np.asarray(M, dtype=np.float64).reshape(-1, 4)
    H = np.asarray(H, dtype=np.float64).reshape(-1, 3)
    d = H[:, None, :] - M[None, :, 1:4]
    r2 = (d * d).sum(-1)
    f = (M[None, :, 0] / r2).sum(1)
    _, g, _ = loss_terms(f)
    G = np.zeros_like(M)
    G[:, 0] = (g[:, None] / r2).sum(0)
    G[:, 1:4] = (g[:, None, None] * 2.0 * M[None, :, 0, None] * d / (r2 * r2)[:, :, None]).sum(0)
    return G


def inside(P, planes, tol=0.0):
    """P [..][3] inside the convex hull: n . p + d <= tol for every plane."""
    P = np.asarray(P, dtype=np.float64)
    pl = np.asarray(planes, dtype=np.float64).reshape(-1, 4)
    s = P @ pl[:, :3].T + pl[:, 3]
    return (s <= tol).all(-1)


def clean(M, planes):
    """Anomaly detection (sec. 2.2): weight zero for control points outside
    the hull (control point overflow) and for negative weights (sign
    abnormality)."""
    M = np.array(M, dtype=np.float64).reshape(-1, 4)
    bad = (M[:, 0] < 0.0) | ~inside(M[:, 1:4], planes)
    M[bad, 0] = 0.0
    return M


def gs(M0, H, planes, E, eta):
    """Alg. GS: E full-batch gradient-descent steps M <- M - eta dL/dM, the
    anomaly cleaning, E more steps.  Returns (M, [L(M0), L after the first
    descent, L at the end])."""
    M = np.array(M0, dtype=np.float64).reshape(-1, 4)
    L0 = gs_loss(M, H)
    for _ in range(E):
        M = M - eta * gs_grad(M, H)
    L1 = gs_loss(M, H)
    M = clean(M, planes)
    for _ in range(E):
        M = M - eta * gs_grad(M, H)
    return M, [L0, L1, gs_loss(M, H)]


# ----------------------------------------------------------- genetic algorithm
def mutate(pop, u, z, C_m, sigma_x, sigma_k):
    """One mutant per individual: gene g changes where u_g < C_m by
    z_g * sigma (sigma_k for weights, sigma_x for coordinates); negative
    weights are set to zero.  pop, u, z: [N_I][n][4]."""
    pop = np.asarray(pop, dtype=np.float64)
    sig = np.array([sigma_k, sigma_x, sigma_x, sigma_x])
    out = pop + np.where(np.asarray(u) < C_m, np.asarray(z, dtype=np.float64) * sig, 0.0)
    out[..., 0] = np.maximum(out[..., 0], 0.0)
    return out


def crossover(pop, perm, C_c):
    """Children of the pairs (perm[2j], perm[2j+1]): control points from
    c = round(C_c n) on are exchanged; child 2j takes the first parent's
    head, child 2j+1 the second's."""
    pop = np.asarray(pop, dtype=np.float64)
    N, n = pop.shape[0], pop.shape[1]
    c = int(np.floor(C_c * n + 0.5))
    kids = np.empty_like(pop)
    for j in range(N // 2):
        a, b = pop[perm[2 * j]], pop[perm[2 * j + 1]]
        kids[2 * j] = np.concatenate([a[:c], b[c:]])
        kids[2 * j + 1] = np.concatenate([b[:c], a[c:]])
    if N % 2:
        kids[N - 1] = pop[perm[N - 1]]
    return kids


def select(pool, F, N):
    """The N individuals of smallest F, ties to the lower pool index."""
    order = np.argsort(np.asarray(F), kind="stable")[:N]
    return np.asarray(pool)[order], np.asarray(F)[order]


def ga(H, pop0, E, C_m, C_c, sigma_x, sigma_k, U, Z, PERM):
    """Alg. GA from the initial population pop0 [N_I][n][4]: per generation
    e, mutation with the draws U[e], Z[e] [N_I][n][4], crossover with the
    pairing PERM[e] [N_I], evaluation, selection of the N_I fittest of
    parents, mutants and children.  Returns the final population (sorted,
    fittest first) and its fitness; the fittest is M^ga."""
    pop = np.asarray(pop0, dtype=np.float64)
    N = pop.shape[0]
    F = np.array([fitness(m, H) for m in pop])
    for e in range(E):
        mut = mutate(pop, U[e], Z[e], C_m, sigma_x, sigma_k)
        kid = crossover(pop, PERM[e], C_c)
        Fm = np.array([fitness(m, H) for m in mut])
        Fk = np.array([fitness(m, H) for m in kid])
        pop, F = select(np.concatenate([pop, mut, kid]), np.concatenate([F, Fm, Fk]), N)
    return pop, F
