"""FP64 oracle of the particle shape descriptors of paper sec. 4: sphericity
Phi, nominal diameter d_n, surface-equivalent-sphere diameter d_s and the
Corey shape factor CSF, for a metaball body C(x) = sum_i k_i/|x - p_i|^2 >= 1
(sec. 2.1, Eq. metaballM).

TEST INFRASTRUCTURE ONLY (like the rest of this package): the tests and the
benchmark's baseline may use it; the product library never does.

Definitions (sec. 4):
  d_n = (6 V / pi)^(1/3)          diameter of the volume-equivalent sphere
  Phi = pi d_n^2 / S              surface of that sphere over the body's
  d_s = sqrt(4 A_p / pi)          diameter of the circle of the projected area
  CSF = d_S / sqrt(d_I d_L)       shortest over the geometric mean of the
                                  intermediate and longest dimensions

Readings (also listed in the design notes):
  - The body's frame is its principal frame (eigenvectors of the inertia
    tensor of the C >= 1 set about its centroid, from the same grid); its
    dimensions d_S <= d_I <= d_L are the extents of the body along those
    three axes.
  - The projected area A_p is the projection onto the plane of the
    intermediate and longest axes (the orientation of largest projection).
  - The paper writes the CSF numerator as d_s; with d_s defined above as a
    projected-area diameter the ratio is not the Corey factor, so the
    numerator is read as the shortest dimension d_S (Corey's definition).

Computation, each step a plain definition on a grid of cell size h over the
box [min p - sqrt(sum k), max p + sqrt(sum k)] (C >= 1 needs some
|x - p_i|^2 <= sum k):
  V     midpoint count of cells with C >= 1 at the cell centre, times h^3
  S     area of the C = 1 surface triangulated by marching tetrahedra (each
        cube split into six tetrahedra along a main diagonal; crossing points
        by linear interpolation of C - 1 along the edges)
  axes  eigenvectors of the inertia tensor of the inside cell centres
  d_*   max - min of the inside cell centres projected on each axis, plus h
  A_p   on a square grid of step h in the plane of the two longer axes
        (-half + h i, half = dimension / 2 + 2 h, i < ceil(2 half / h) + 1
        on each axis, about the centroid): columns along the shortest axis,
        sampled the same way, with at least one sample with C >= 1; their
        count times h^2
"""
from __future__ import annotations

import numpy as np


def metaball(cp, k, x):
    """C at the points x [..][3]."""
    d2 = ((np.asarray(x)[..., None, :] - np.asarray(cp)) ** 2).sum(-1)
    with np.errstate(divide="ignore"):
        return (np.asarray(k) / d2).sum(-1)


def _box(cp, k, h):
    cp = np.asarray(cp, dtype=np.float64).reshape(-1, 3)
    r = np.sqrt(np.sum(k))
    lo = cp.min(0) - r - h
    hi = cp.max(0) + r + h
    n = np.ceil((hi - lo) / h).astype(int) + 1
    return lo, n


def volume_cells(cp, k, h):
    """Centres of the cells with C >= 1 (midpoint rule) and V = count h^3."""
    lo, n = _box(cp, k, h)
    axes = [lo[a] + h * (np.arange(n[a]) + 0.5) for a in range(3)]
    pts = []
    for zc in axes[2]:
        X, Y = np.meshgrid(axes[0], axes[1], indexing="ij")
        P = np.stack([X, Y, np.full_like(X, zc)], -1).reshape(-1, 3)
        inside = metaball(cp, k, P) >= 1.0
        pts.append(P[inside])
    P = np.concatenate(pts)
    return P, len(P) * h ** 3


# the six tetrahedra of a cube (corner indices 0..7 with bit a = offset on
# axis a), all sharing the diagonal 0 - 7
_TETS = np.array([[0, 1, 3, 7], [0, 3, 2, 7], [0, 2, 6, 7], [0, 6, 4, 7], [0, 4, 5, 7], [0, 5, 1, 7]])
_CORNER = np.array([[(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.float64)


def _tet_area(P, g):
    """Area of the g = 0 surface inside tetrahedra P [T][4][3] with values g
    [T][4] (linear interpolation): one triangle (one or three corners
    positive) or a quadrilateral (two)."""
    pos = g >= 0.0
    npos = pos.sum(1)
    area = np.zeros(len(g))

    def cut(a, b, ia, ib):
        t = (g[ia, a] / (g[ia, a] - g[ia, b]))[:, None]
        return P[ia, a] + t * (P[ia, b] - P[ia, a])

    for m in (1, 3):
        sel = np.flatnonzero(npos == m)
        if len(sel) == 0:
            continue
        lone = np.where(pos[sel], 1, 0) if m == 1 else np.where(pos[sel], 0, 1)
        a = np.argmax(lone, axis=1)  # the corner on its own side
        others = np.array([[j for j in range(4) if j != aa] for aa in a])
        q = [cut(a, others[:, j], sel, sel) for j in range(3)]
        area[sel] = 0.5 * np.linalg.norm(np.cross(q[1] - q[0], q[2] - q[0]), axis=1)
    sel = np.flatnonzero(npos == 2)
    if len(sel):
        order = np.argsort(~pos[sel], axis=1, kind="stable")  # two positive first
        p0, p1, m0, m1 = order[:, 0], order[:, 1], order[:, 2], order[:, 3]
        a = cut(p0, m0, sel, sel)
        b = cut(p0, m1, sel, sel)
        c = cut(p1, m1, sel, sel)
        d = cut(p1, m0, sel, sel)
        area[sel] = 0.5 * (np.linalg.norm(np.cross(b - a, c - a), axis=1)
                           + np.linalg.norm(np.cross(c - a, d - a), axis=1))
    return area


def surface_area(cp, k, h):
    """Area of the C = 1 surface, marching tetrahedra on the grid of step h."""
    lo, n = _box(cp, k, h)
    xs = [lo[a] + h * np.arange(n[a]) for a in range(3)]
    X, Y = np.meshgrid(xs[0], xs[1], indexing="ij")
    total = 0.0
    prev = metaball(cp, k, np.stack([X, Y, np.full_like(X, xs[2][0])], -1)) - 1.0
    for iz in range(1, n[2]):
        cur = metaball(cp, k, np.stack([X, Y, np.full_like(X, xs[2][iz])], -1)) - 1.0
        # corner values of the cells between planes iz-1 and iz
        g = np.stack([prev[:-1, :-1], prev[1:, :-1], prev[:-1, 1:], prev[1:, 1:],
                      cur[:-1, :-1], cur[1:, :-1], cur[:-1, 1:], cur[1:, 1:]], -1).reshape(-1, 8)
        mixed = (g.min(1) < 0.0) & (g.max(1) >= 0.0)
        if mixed.any():
            gi = g[mixed]
            ii, jj = np.nonzero(mixed.reshape(n[0] - 1, n[1] - 1))
            org = np.stack([xs[0][ii], xs[1][jj], np.full(len(ii), xs[2][iz - 1])], 1)
            corners = org[:, None, :] + h * _CORNER[None]
            Pt = corners[:, _TETS].reshape(-1, 4, 3)
            gt = gi[:, _TETS].reshape(-1, 4)
            total += _tet_area(Pt, gt).sum()
        prev = cur
    return float(total)


def principal_frame(P):
    """Centroid and principal axes (columns, by increasing extent) of the
    inside cell centres P, with the extents along them.  Each axis is signed
    so that its component of largest magnitude is positive (a convention
    that makes the projection grid below unique)."""
    c = P.mean(0)
    r = P - c
    I = np.eye(3) * (r * r).sum() - r.T @ r  # per unit mass and cell volume
    _, vec = np.linalg.eigh(I)
    for j in range(3):
        if vec[np.argmax(np.abs(vec[:, j])), j] < 0:
            vec[:, j] = -vec[:, j]
    proj = r @ vec
    ext = proj.max(0) - proj.min(0)
    order = np.argsort(ext, kind="stable")
    return c, vec[:, order], ext[order]


def projected_area(cp, k, h, c, axes, ext):
    """Area of the projection onto the plane of the two longer axes: columns
    along the shortest axis with at least one sample inside."""
    aS, aI, aL = axes[:, 0], axes[:, 1], axes[:, 2]
    half = 0.5 * ext + 2 * h
    cnt = np.ceil(2 * half / h).astype(int) + 1
    u = -half[2] + h * np.arange(cnt[2])
    v = -half[1] + h * np.arange(cnt[1])
    w = -half[0] + h * np.arange(cnt[0])
    U, Vv = np.meshgrid(u, v, indexing="ij")
    hit = np.zeros(U.shape, dtype=bool)
    for ww in w:
        P = c + U[..., None] * aL + Vv[..., None] * aI + ww * aS
        hit |= metaball(cp, k, P) >= 1.0
    return float(hit.sum()) * h * h


def descriptors(cp, k, h=0.25):
    """V, S, A_p, the dimensions (d_S, d_I, d_L) and Phi, d_n, d_s, CSF."""
    P, V = volume_cells(cp, k, h)
    S = surface_area(cp, k, h)
    c, axes, ext = principal_frame(P)
    dims = ext + h
    Ap = projected_area(cp, k, h, c, axes, dims)
    dn = (6.0 * V / np.pi) ** (1.0 / 3.0)
    ds = np.sqrt(4.0 * Ap / np.pi)
    return {"V": V, "S": S, "A_p": Ap, "dims": dims, "d_n": dn, "d_s": ds,
            "Phi": np.pi * dn * dn / S, "CSF": dims[0] / np.sqrt(dims[1] * dims[2]), "centroid": c, "axes": axes}
