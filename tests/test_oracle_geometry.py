"""Pins of the oracle's metaball geometry: flags, cut links, link fractions q
and body properties (paper sec. 2.1, Eq. metaballM: C(x) = sum k_i/|x - p_i|^2,
C = 1 on the surface, C > 1 inside; sec. 2.3.2: q solves C(x_f + q e) = c_0,
read with c_0 = 1 along the link towards the solid node).

Pins: a single control point is a sphere of radius sqrt(k), so flags are
lattice points of a ball (2109 for radius 8: the count of integer points
with x^2 + y^2 + z^2 <= 64) and q is the smaller root of a quadratic; two equal
control points at +-a reach x* = sqrt(a^2 + k + sqrt(k^2 + 4 k a^2)) on their
axis; general bodies are checked by brute-force numpy evaluation."""
import itertools

import numpy as np
import pytest

import oracle
import workloads


def d3q19_dirs():
    return [e for e in itertools.product((-1, 0, 1), repeat=3) if 0 < sum(x * x for x in e) <= 2]


def brute_flags(cfg, cps_list):
    """Owner per node by direct numpy evaluation (lowest index with C >= 1)."""
    z, y, x = np.meshgrid(np.arange(cfg.nz), np.arange(cfg.ny), np.arange(cfg.nx), indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(float)
    L = np.array([cfg.nx, cfg.ny, cfg.nz], float)
    per = np.array([(cfg.periodic >> a) & 1 for a in range(3)], bool)
    own = np.full(len(pts), -1, np.int32)
    Cvals = []
    for p, (lab, k) in enumerate(cps_list):
        C = np.zeros(len(pts))
        for c, kk in zip(lab, k):
            d = pts - c
            d[:, per] -= L[per] * np.floor(d[:, per] / L[per] + 0.5)
            C += kk / (d * d).sum(1)
        own[(own < 0) & (C >= 1.0)] = p
        Cvals.append(C)
    return own, Cvals


def brute_links(cfg, own):
    """Cut links (node, direction vector) by direct enumeration: fluid node x
    and direction e with x - e an in-domain solid node."""
    solid = (own >= 0).reshape(cfg.nz, cfg.ny, cfg.nx)
    links = []
    for e in d3q19_dirs():
        ex, ey, ez = e
        src = np.roll(solid, shift=(ez, ey, ex), axis=(0, 1, 2))  # src[x] = solid[x - e]
        cut = (~solid) & src
        for n in np.flatnonzero(cut.ravel()):
            links.append((int(n), e))
    return links


@pytest.mark.parametrize("center,counts", [("integer", (2109, 4530, 1178)),
                                           ("half", (2176, 4704, 1200))])
def test_sphere_flags_and_links(center, counts):
    cfg = workloads.config1(center=center)
    o = oracle.Oracle(cfg)
    own = o.owner()
    lab, k = o.cps(0)
    own_b, _ = brute_flags(cfg, [(lab, k)])
    assert np.array_equal(own, own_b)
    assert (own >= 0).sum() == counts[0]
    node, d, ow, q = o.links()
    assert len(node) == counts[1]
    assert len(np.unique(node)) == counts[2]
    e, _, _ = oracle.lattice()
    got = sorted((int(n), tuple(int(v) for v in e[i])) for n, i in zip(node, d))
    assert got == sorted(brute_links(cfg, own_b))
    assert np.all(ow == 0)


def test_sphere_ties_exact():
    """k = 64 at an integer node: the 6 nodes at distance 8 on the axes have
    C = 1 exactly and are solid."""
    cfg = workloads.config1()
    o = oracle.Oracle(cfg)
    own = o.owner().reshape(64, 64, 64)
    for dx, dy, dz in [(8, 0, 0), (-8, 0, 0), (0, 8, 0), (0, -8, 0), (0, 0, 8), (0, 0, -8)]:
        assert own[32 + dz, 32 + dy, 32 + dx] == 0
        assert own[32 + int(np.sign(dz)) * (abs(dz) + 1) if dz else 32,
                   32 + int(np.sign(dy)) * (abs(dy) + 1) if dy else 32,
                   32 + int(np.sign(dx)) * (abs(dx) + 1) if dx else 32] == -1


@pytest.mark.parametrize("center", ["integer", "half"])
def test_sphere_q_closed_form(center):
    """|x_f - s e - p|^2 = k: q = [d.e - sqrt((d.e)^2 - |e|^2(|d|^2 - k))]/|e|^2."""
    cfg = workloads.config1(center=center)
    o = oracle.Oracle(cfg)
    node, d, ow, q = o.links()
    e, _, _ = oracle.lattice()
    p = np.array(cfg.particles[0].x)
    k = cfg.particles[0].cp_k[0]
    xf = np.stack([node % 64, (node // 64) % 64, node // 4096], 1).astype(float)
    ev = e[d].astype(float)
    dd = xf - p
    de = (dd * ev).sum(1)
    ee = (ev * ev).sum(1)
    disc = de * de - ee * ((dd * dd).sum(1) - k)
    qa = (de - np.sqrt(disc)) / ee
    assert np.all((q > 0) & (q <= 1))
    # well-conditioned links to 1e-13; links tangent to the sphere (double
    # root, disc = 0) are resolved only to sqrt(FP64 epsilon)
    good = disc > 1e-3
    assert good.sum() > 0.9 * len(q)
    assert np.abs(q - qa)[good].max() < 1e-13
    assert np.abs(q - qa).max() < 2e-7


def test_two_point_axial_extent():
    """Two equal control points at c +- a x: C = 1 on the axis at
    x* = sqrt(a^2 + k + sqrt(k^2 + 4 k a^2)) from c."""
    a, k, n = 3.0, 16.0, 40
    c = np.array([20.0, 20.0, 20.0])
    cfg = workloads.Config(nx=n, ny=n, nz=n, periodic=7, tau=0.8, bc=workloads.BC_IBB,
                           particles=[workloads.Particle(cp_xyz=np.array([[-a, 0, 0], [a, 0, 0]]),
                                                         cp_k=np.array([k, k]), x=c, density=1.0,
                                                         mode=workloads.MODE_KINEMATIC)])
    o = oracle.Oracle(cfg)
    xs = np.sqrt(a * a + k + np.sqrt(k * k + 4 * k * a * a))
    xf = int(np.floor(c[0] + xs)) + 1  # first fluid node beyond the tip on +x
    e, _, _ = oracle.lattice()
    i_plus = [i for i in range(19) if tuple(e[i]) == (1, 0, 0)][0]
    node, d, ow, q = o.links()
    n_f = xf + n * (20 + n * 20)
    sel = (node == n_f) & (d == i_plus)
    assert sel.sum() == 1
    assert q[sel][0] == pytest.approx(xf - (c[0] + xs), abs=1e-13)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_general_body_flags_and_q(seed):
    """Random 8-point body: flags match brute force; every link's q is a root
    (C(x_w) = 1 to 1e-12) and no sampled point between x_f and x_w is solid."""
    off, k = workloads.random_body(np.random.Generator(np.random.PCG64(seed)), 8, 6.0)
    cfg = workloads.Config(nx=40, ny=40, nz=40, periodic=7, tau=0.8, bc=workloads.BC_IBB,
                           particles=[workloads.Particle(cp_xyz=off, cp_k=k,
                                                         x=np.array([20.3, 19.6, 20.1]),
                                                         density=1.0,
                                                         mode=workloads.MODE_KINEMATIC)])
    o = oracle.Oracle(cfg)
    lab, kk = o.cps(0)
    own_b, (C,) = brute_flags(cfg, [(lab, kk)])
    own = o.owner()
    assert np.array_equal(own, own_b)
    assert np.abs(C - 1.0).min() > 1e-9  # no near-ties, so the comparison is meaningful
    node, d, ow, q = o.links()
    e, _, _ = oracle.lattice()
    xf = np.stack([node % 40, (node // 40) % 40, node // 1600], 1).astype(float)
    xw = xf - q[:, None] * e[d]
    Cw = np.array([oracle.metaball_eval(lab, kk, x) for x in xw])
    assert np.abs(Cw - 1).max() < 1e-12
    for s in np.linspace(0, 1, 33)[:-1]:
        pts = xf - (s * q)[:, None] * e[d]
        Cs = np.array([oracle.metaball_eval(lab, kk, x) for x in pts])
        assert np.all(Cs < 1.0 + 1e-12)


def test_body_properties_sphere():
    """Sphere of radius sqrt(k): V = 4/3 pi k^1.5, I = 2/5 V k per unit
    density, centroid at the control point (midpoint rule, h = 1/8)."""
    k = 64.0
    V, c, I, cnt = oracle.body_properties(np.array([[1.5, -2.0, 3.25]]), np.array([k]), 0.125)
    Vt = 4 / 3 * np.pi * k ** 1.5
    assert V == pytest.approx(Vt, rel=2e-3)
    assert np.array_equal(c, np.array([1.5, -2.0, 3.25]))
    assert np.allclose(np.diag(I), 0.4 * Vt * k, rtol=3e-3)
    assert np.abs(I - np.diag(np.diag(I))).max() < 1e-9 * I.max()


def test_body_properties_two_spheres_far():
    """Two far-apart control points: each acts alone to leading order, so V is
    twice a sphere's and the centroid is the k-weighted... midpoint for equal k."""
    k = 9.0
    V, c, I, cnt = oracle.body_properties(np.array([[-20.0, 0, 0], [20.0, 0, 0]]),
                                          np.array([k, k]), 0.125)
    # far field of the other point adds ~k/40^2 to C, enlarging each ball slightly
    assert V == pytest.approx(2 * 4 / 3 * np.pi * k ** 1.5, rel=2e-2)
    assert np.allclose(c, [0, 0, 0], atol=1e-12)
    # parallel-axis theorem: I_yy ~ 2 (2/5 v k + v 20^2)
    v = V / 2
    assert I[1, 1] == pytest.approx(2 * (0.4 * v * k + v * 400.0), rel=2e-2)


@pytest.mark.parametrize("rs", [0.5, 1.5, 3.0])
def test_sphero_metaball_level_keeps_a_sphere(rs):
    """Sec. 2.3.2 (q solves f = c_0, c_0 depending on R_s), read with the
    sphero-metaball's inner body (the body scaled by s = 1 - R_s/sqrt(k)
    about its centre, weights s^2 k) at c_0 = s^2: for one control point the
    inner ball of radius s sqrt(k) dilated by R_s is the ball itself, so the
    link fractions equal the C = 1 closed form for every R_s."""
    cfg = workloads.config1()
    cfg.contact_rs, cfg.link_c0 = rs, 1
    o = oracle.Oracle(cfg)
    node, d, ow, q = o.links()
    e, _, _ = oracle.lattice()
    p = np.array(cfg.particles[0].x)
    k = cfg.particles[0].cp_k[0]
    xf = np.stack([node % 64, (node // 64) % 64, node // 4096], 1).astype(float)
    ev = e[d].astype(float)
    dd = xf - p
    de = (dd * ev).sum(1)
    ee = (ev * ev).sum(1)
    disc = de * de - ee * ((dd * dd).sum(1) - k)
    qa = (de - np.sqrt(disc)) / ee
    good = disc > 1e-3
    assert len(q) == 4530
    assert np.abs(q - qa)[good].max() < 1e-12
    assert np.abs(q - qa).max() < 2e-7


@pytest.mark.parametrize("seed", [1, 2])
def test_sphero_metaball_level_general_body(seed):
    """An 8-point body with R_s = 1: each q in (0, 1) is a root of the inner
    body's level equation sum s^2 k / |x_w - X - s (p - X)|^2 = s^2 (to 1e-12),
    with no sample between x_f and x_w at or above the level; q = 1 only where
    the solid node is below the level, and q -> 0 only where x_f is at or above
    it (the two surfaces differ for a non-spherical body)."""
    off, k = workloads.random_body(np.random.Generator(np.random.PCG64(seed)), 8, 6.0)
    cfg = workloads.Config(nx=40, ny=40, nz=40, periodic=7, tau=0.8, bc=workloads.BC_IBB, contact_rs=1.0,
                           link_c0=1,
                           particles=[workloads.Particle(cp_xyz=off, cp_k=k, x=np.array([20.3, 19.6, 20.1]),
                                                         density=1.0, mode=workloads.MODE_KINEMATIC)])
    o = oracle.Oracle(cfg)
    lab, kk = o.cps(0)
    X = o.particle(0)["x"]
    s = 1.0 - 1.0 / np.sqrt(kk.sum())
    inner, kin = X + s * (lab - X), s * s * kk
    node, d, ow, q = o.links()
    e, _, _ = oracle.lattice()
    xf = np.stack([node % 40, (node // 40) % 40, node // 1600], 1).astype(float)
    ev = e[d].astype(float)

    def f(x):
        return oracle.metaball_eval(inner, kin, x)

    mid = (q > 1e-9) & (q < 1.0)
    assert mid.sum() > 0.5 * len(q)
    for j in np.flatnonzero(mid)[::7]:
        assert abs(f(xf[j] - q[j] * ev[j]) - s * s) < 1e-12
        for t in np.linspace(0, 1, 33)[:-1]:
            assert f(xf[j] - t * q[j] * ev[j]) < s * s * (1 + 1e-12)
    for j in np.flatnonzero(q >= 1.0):
        assert all(f(xf[j] - t * ev[j]) < s * s for t in np.arange(1, 9) / 8)
    for j in np.flatnonzero(q <= 1e-9):
        assert f(xf[j] - (1 / 8) * ev[j]) >= s * s


def _scan_links(cfg, m=64, chunk=20000):
    """For every cut link of the oracle's initial state: the index J of the
    first of m equal samples s = j/m along the link (towards the solid node)
    with C >= 1, and the number of in/out changes among the samples inside
    the eighth of the link that holds sample J."""
    o = oracle.Oracle(cfg)
    node, d, own, q = o.links()
    e, _, _ = oracle.lattice()
    L = np.array([cfg.nx, cfg.ny, cfg.nz], float)
    per = np.array([(cfg.periodic >> a) & 1 for a in range(3)], bool)
    xf = np.stack([node % cfg.nx, (node // cfg.nx) % cfg.ny, node // (cfg.nx * cfg.ny)], 1).astype(float)
    ev = e[d].astype(float)
    s = np.arange(1, m + 1) / m
    first = np.full(len(node), -1)
    changes = np.zeros(len(node), int)
    for p in range(len(cfg.particles)):
        lab, k = o.cps(p)
        idx = np.nonzero(own == p)[0]
        for c0 in range(0, len(idx), chunk):
            sel = idx[c0:c0 + chunk]
            r = xf[sel, None, None, :] - s[None, :, None, None] * ev[sel, None, None, :] - lab[None, None]
            r[..., per] -= L[per] * np.floor(r[..., per] / L[per] + 0.5)
            inside = (k / (r * r).sum(-1)).sum(-1) >= 1.0
            J = np.where(inside.any(1), inside.argmax(1) + 1, -1)
            first[sel] = J
            lo = (J - 1) // (m // 8) * (m // 8)            # samples lo+1 .. lo+m/8 form J's eighth
            j = np.arange(1, m + 1)
            prev = np.concatenate([np.zeros((len(sel), 1), bool), inside[:, :-1]], 1)
            ineighth = (j[None] > lo[:, None]) & (j[None] <= lo[:, None] + m // 8)
            changes[sel] = (ineighth & (inside != prev)).sum(1)
    return q, first, changes


@pytest.mark.parametrize("case", ["settling", "two_bodies", "suspension", "dkt_a4"])
def test_eight_sample_bracket_against_a_finer_scan(case):
    """Link fraction as the FIRST root (sec. 2.3.2, reading of the bracket
    with 8 samples): on the bodies of the benchmark workloads at their sizes
    (settling body 128x128x384, two bodies 160x160x640, the 200-body
    suspension at 96^3 with its volume fraction, the most elongated DKT
    body), a scan with 64 samples per link finds every link's first solid
    sample in the sixty-fourth that holds q, so no thin part of a body that a
    link crosses before its root is missed, and inside q's eighth the samples
    change between fluid and solid only once (the bisection has one root to
    find).  The same count on the full 256^3 suspension (1 446 154 links) is
    zero as well."""
    if case == "settling":
        cfg = workloads.config2()
    elif case == "two_bodies":
        cfg = workloads.config3()
    elif case == "suspension":
        cfg = workloads.config5(n_bodies=10, box=96)
    else:
        cfg = workloads.dkt_pair(*workloads.dkt_body(4.0))
    q, J, changes = _scan_links(cfg)
    assert len(q) > 1000
    assert (J > 0).all()
    assert np.all(q > (J - 1) / 64 - 1e-12) and np.all(q <= J / 64 + 1e-12)
    assert (changes == 1).all()
