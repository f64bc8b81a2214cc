"""Pins of the oracle's contact model (paper sec. 2.3.1: sphero-metaball
contact, Newton-Raphson for the stationary point of f0 + f1 (Eq. eq:grad),
Taylor projection to the closest points (Eq. eq:cp), contact properties
(Eqs. eq:contactprop, eq:contactprop2), linear spring-dashpot with Coulomb
friction).

- two single-point spheres: the stationary point divides the centre segment
  in the ratio (k0'/k1')^(1/3) of the inner weights (exact);
- the Taylor-projected closest point lies within 1.5 r' eps^2 of the exact one
  (eps = relative distance of x_m from the inner surface), so delta converges
  to R0 + R1 - D quadratically as the spheres close in;
- head-on collision of two spheres reproduces the restitution coefficient;
- a sphere resting on a wall settles at delta = (m - rho0 V) g / k_n;
- a sphere launched sliding on a wall ends rolling without slipping at
  v = v0 / (1 + I/(m a^2)) (5/7 v0 for a solid sphere with a = R), whatever
  mu is."""
import numpy as np
import pytest

import oracle
import workloads


def two_spheres(k0, k1, D, rs=1.0, n=48, v0=(0, 0, 0), v1=(0, 0, 0), kn=1.0, en=0.5, n_sub=1,
                periodic=7, mode=workloads.MODE_FREE):
    c = np.array([n / 2 - D / 2, n / 2 + 0.1, n / 2 - 0.2])
    P0 = workloads.Particle(cp_xyz=np.zeros((1, 3)), cp_k=np.array([k0]), x=c.copy(), v=np.array(v0, float),
                            density=1.0, mode=mode)
    P1 = workloads.Particle(cp_xyz=np.zeros((1, 3)), cp_k=np.array([k1]), x=c + [D, 0, 0],
                            v=np.array(v1, float), density=1.0, mode=mode)
    cfg = workloads.Config(nx=n, ny=n, nz=n, periodic=periodic, tau=0.8, n_sub=n_sub, particles=[P0, P1],
                           contact_rs=rs, contact_kn=kn, contact_en=en, contact_mu=0.5, quad_h=0.25)
    return cfg


@pytest.mark.parametrize("k0,k1", [(16.0, 16.0), (16.0, 36.0), (49.0, 9.0)])
def test_stationary_point_ratio(k0, k1):
    D = np.sqrt(k0) + np.sqrt(k1) + 0.5
    o = oracle.Oracle(two_spheres(k0, k1, D))
    r, xm, xc0, xc1, xcp, n, delta = o.pair_geometry(0, 1)
    X0, X1 = o.particle(0)["x"], o.particle(1)["x"]
    s0, s1 = 1 - 1 / np.sqrt(k0), 1 - 1 / np.sqrt(k1)
    ratio = (s0 ** 2 * k0 / (s1 ** 2 * k1)) ** (1 / 3)
    expect = X0 + (X1 - X0) * ratio / (1 + ratio)
    assert r >= 0
    assert np.abs(xm - expect).max() < 1e-10
    assert np.allclose(n, (X0 - X1) / np.linalg.norm(X0 - X1), atol=1e-12)


def test_taylor_projection_is_second_order():
    """Equal spheres (k = 25, inner radius r' = 4): x_m sits at d = r'(1 + eps)
    from each centre; the Taylor point lands at r'(1 - 1.5 eps^2 - 0.5 eps^3)
    from the centre (exact for f = k'/d^2), so delta = 2R - D - 2 r'(1.5 eps^2 +
    0.5 eps^3)."""
    k, rp = 25.0, 4.0
    errs = []
    for gap in (0.8, 0.4, 0.2, 0.1):
        D = 2 * rp + 2 * gap
        eps = gap / rp
        o = oracle.Oracle(two_spheres(k, k, D))
        r, xm, xc0, xc1, xcp, n, delta = o.pair_geometry(0, 1)
        X0 = o.particle(0)["x"]
        exact_c0 = X0 + rp * (xm - X0) / np.linalg.norm(xm - X0)
        e = np.linalg.norm(xc0 - exact_c0)
        assert e == pytest.approx(rp * (1.5 * eps ** 2 + 0.5 * eps ** 3), rel=1e-9)
        assert delta == pytest.approx(2 * 5.0 - D - 2 * rp * (1.5 * eps ** 2 + 0.5 * eps ** 3), abs=1e-11)
        assert np.allclose(xcp, 0.5 * (xc0 + xc1), atol=1e-12)  # symmetric contact point
        errs.append(e)
    assert errs[-1] < errs[0] / 50  # quadratic in eps


def test_head_on_restitution():
    """Linear spring-dashpot: e = exp(-pi zeta / sqrt(1 - zeta^2)).  The
    Taylor projection stiffens the spring by about (1 + 3 R_s/r'), so the pin
    uses R_s/r' ~ 0.013 (R = 8, R_s = 0.1) where that is below 1 %."""
    en, vr = 0.5, 0.02
    cfg = two_spheres(64.0, 64.0, 16.0 + 0.5, rs=0.1, kn=480.0, en=en, n_sub=20,
                      v0=(vr / 2, 0, 0), v1=(-vr / 2, 0, 0), n=48)
    o = oracle.Oracle(cfg)
    o.dem_only(80)
    v0, v1 = o.particle(0)["v"], o.particle(1)["v"]
    assert o.n_contacts > 0 and o.n_contact_fail == 0
    e_meas = (v1[0] - v0[0]) / vr
    assert e_meas == pytest.approx(en, rel=0.02)
    assert abs(v0[0] + v1[0]) < 1e-12  # momentum conserved (equal masses)


def sphere_on_floor(v0=(0.0, 0.0, 0.0), mu=0.5, kn=5.0, g=2e-4, n_sub=20):
    k = 16.0  # R = 4
    P = workloads.Particle(cp_xyz=np.zeros((1, 3)), cp_k=np.array([k]), x=np.array([20.0, 20.0, 3.5]),
                           v=np.array(v0, float), density=3.0)
    return workloads.Config(nx=60, ny=40, nz=20, periodic=workloads.PERIODIC_X | workloads.PERIODIC_Y,
                            tau=0.8, n_sub=n_sub, g_particle=np.array([0.0, 0.0, -g]), particles=[P],
                            contact_rs=1.0, contact_kn=kn, contact_en=0.3, contact_mu=mu, quad_h=0.125)


def test_sphere_resting_on_wall():
    cfg = sphere_on_floor()
    o = oracle.Oracle(cfg)
    o.dem_only(3000)
    P = o.particle(0)
    weight = (P["m"] - P["V"]) * 2e-4
    r, xcw, xcm, xcp, n, delta = o.wall_geometry(0, 2, 0)
    assert r == 1
    assert np.allclose(n, [0, 0, 1], atol=1e-9)
    assert delta == pytest.approx(weight / cfg.contact_kn, rel=1e-3)
    # sphere (inner radius r' = 3): the Taylor step from the wall plane covers
    # exactly r'(eps + 1.5 eps^2 + 0.5 eps^3), eps = (d - r')/r', d = centre-plane distance
    rp, d = 3.0, P["x"][2] + 0.5
    eps = (d - rp) / rp
    assert delta == pytest.approx(1.0 - rp * (eps + 1.5 * eps ** 2 + 0.5 * eps ** 3), abs=1e-10)
    assert np.allclose(xcw[:2], P["x"][:2], atol=1e-10)  # foot of the centre on the plane
    assert abs(P["v"][2]) < 1e-7


@pytest.mark.parametrize("mu", [0.2, 0.6])
def test_sliding_sphere_ends_rolling(mu):
    v0 = 0.01
    o = oracle.Oracle(sphere_on_floor(mu=mu))
    o.dem_only(3000)  # settle at rest on the floor first, then launch it sliding
    P = o.particle(0)
    o.set_particle_state(0, P["x"], P["quat"], [v0, 0, 0], [0, 0, 0])
    o.dem_only(4000)
    P = o.particle(0)
    # friction and the normal force act at the contact point below the centre
    # and gravity through the centre, so m v a + I w is conserved about the
    # contact line (a = centre height above the contact point); rolling without
    # slipping (v = w a) then gives v = v0 / (1 + I/(m a^2)) (5/7 v0 when a = R)
    r, xcw, xcm, xcp, n, delta = o.wall_geometry(0, 2, 0)
    arm = P["x"][2] - xcp[2]
    assert P["omega"][1] * arm == pytest.approx(P["v"][0], rel=1e-3)
    assert P["v"][0] == pytest.approx(v0 / (1 + P["I"][1, 1] / (P["m"] * arm ** 2)), rel=2e-3)
    assert 0.66 * v0 < P["v"][0] < 5 / 7 * v0
