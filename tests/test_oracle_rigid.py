"""Pins of the oracle's rigid-body update (paper sec. 2.3.1: m a = F,
d(I w)/dt = T; the integrator is the reading: semi-implicit Euler in
n_sub sub-steps, body-frame Euler equation, exact rotation per sub-step).

- constant force: v_m = v0 + m a dt, x_m = x0 + m v0 dt + a dt^2 m(m+1)/2
  over m sub-steps of dt = 1/n_sub (semi-implicit Euler, exact);
- weight minus buoyancy (m - rho0 V) g;
- torque-free spin about a principal axis keeps w and rotates the body by
  exactly |w| t (the principal axis found with numpy.linalg.eigh);
- the quaternion stays a unit quaternion;
- from rest, one sub-step under a torque T gives w = I_lab^-1 T dt with
  I_lab = R I_body R^T (Euler's equation with w = 0), and the body turns
  about w by |w| dt (Rodrigues' rotation of its control points)."""
import numpy as np
import pytest

import oracle
import workloads


def make(off, k, mode=workloads.MODE_FREE, n_sub=1, gp=(0, 0, 0), density=2.0):
    p = workloads.Particle(cp_xyz=off, cp_k=k, x=np.array([20.0, 20.0, 20.0]),
                           density=density, mode=mode)
    cfg = workloads.Config(nx=40, ny=40, nz=40, periodic=7, tau=0.8, n_sub=n_sub,
                           g_particle=np.array(gp, float), particles=[p])
    return oracle.Oracle(cfg)


def quat_rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


@pytest.mark.parametrize("n_sub", [1, 4, 100])
def test_constant_force_closed_form(n_sub):
    o = make(np.zeros((1, 3)), np.array([16.0]), n_sub=n_sub)
    P = o.particle(0)
    F = np.array([1e-3, -2e-3, 5e-4])
    a = F / P["m"]
    x0, v0 = P["x"].copy(), np.array([0.01, 0.0, -0.02])
    o.set_particle_state(0, x0, P["quat"], v0, np.zeros(3))
    for n in range(1, 21):
        o.rigid_body_step(0, F, np.zeros(3))
        m, dt = n * n_sub, 1.0 / n_sub
        P = o.particle(0)
        assert np.allclose(P["v"], v0 + m * a * dt, rtol=1e-12, atol=1e-16)
        assert np.allclose(P["x"], x0 + m * v0 * dt + a * dt * dt * m * (m + 1) / 2,
                           rtol=1e-13, atol=1e-12)


def test_weight_minus_buoyancy():
    g = np.array([0.0, 0.0, -2e-5])
    o = make(np.zeros((1, 3)), np.array([16.0]), gp=g, density=1.5)
    P = o.particle(0)
    o.rigid_body_step(0, np.zeros(3), np.zeros(3))
    v = o.particle(0)["v"]
    assert np.allclose(v, (P["m"] - 1.0 * P["V"]) * g / P["m"], rtol=1e-14)
    assert P["m"] == pytest.approx(1.5 * P["V"], rel=1e-15)


def test_torque_free_spin_about_principal_axis():
    off, k = workloads.random_body(np.random.Generator(np.random.PCG64(7)), 6, 5.0)
    o = make(off, k)
    P = o.particle(0)
    evals, evecs = np.linalg.eigh(P["I"])
    axis = evecs[:, 0]
    w0 = 0.01 * axis
    o.set_particle_state(0, P["x"], np.array([1.0, 0, 0, 0]), np.zeros(3), w0)
    for n in range(1, 51):
        o.rigid_body_step(0, np.zeros(3), np.zeros(3))
    P = o.particle(0)
    assert np.allclose(P["omega"], w0, atol=1e-15)
    ang = 0.01 * 50
    qe = np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * axis])
    assert np.allclose(P["quat"], qe, atol=1e-13) or np.allclose(P["quat"], -qe, atol=1e-13)
    assert np.linalg.norm(P["quat"]) == pytest.approx(1.0, abs=1e-15)


def test_asymmetric_top_conserves_angular_momentum_norm_to_first_order():
    """Torque-free asymmetric top off its principal axes: |L| = |I w_b| is
    an exact invariant of the Euler equation; the explicit update keeps it
    to O(dt) over unit time, and the error falls with n_sub."""
    off, k = workloads.random_body(np.random.Generator(np.random.PCG64(8)), 6, 5.0)
    errs = []
    for n_sub in (1, 4):
        o = make(off, k, n_sub=n_sub)
        P = o.particle(0)
        w0 = np.array([0.02, 0.015, -0.01])
        o.set_particle_state(0, P["x"], np.array([1.0, 0, 0, 0]), np.zeros(3), w0)
        L0 = np.linalg.norm(P["I"] @ w0)
        for _ in range(100):
            o.rigid_body_step(0, np.zeros(3), np.zeros(3))
        P = o.particle(0)
        R = quat_rot(P["quat"])
        Lb = P["I"] @ (R.T @ P["omega"])
        errs.append(abs(np.linalg.norm(Lb) / L0 - 1))
        assert np.linalg.norm(P["quat"]) == pytest.approx(1.0, abs=1e-14)
    assert errs[0] < 2e-3
    assert errs[1] < errs[0] / 2.5


def test_kinematic_body_moves_with_given_velocity():
    o = make(np.zeros((1, 3)), np.array([16.0]), mode=workloads.MODE_KINEMATIC)
    P = o.particle(0)
    v, w = np.array([0.01, 0.02, -0.03]), np.array([0.0, 0.0, 0.05])
    o.set_particle_state(0, P["x"], P["quat"], v, w)
    for _ in range(10):
        o.rigid_body_step(0, np.array([1.0, 1, 1]), np.array([1.0, 1, 1]))
    Q = o.particle(0)
    assert np.allclose(Q["x"], P["x"] + 10 * v, rtol=1e-14)
    assert np.allclose(Q["quat"], [np.cos(0.25), 0, 0, np.sin(0.25)], atol=1e-14)


def rodrigues(axis_angle, v):
    th = np.linalg.norm(axis_angle)
    kx = axis_angle / th
    return (v * np.cos(th) + np.cross(kx, v) * np.sin(th)
            + np.outer(v @ kx, kx) * (1 - np.cos(th)))


@pytest.mark.parametrize("n_sub", [1, 3])
def test_applied_torque_from_rest(n_sub):
    """Asymmetric body at a general orientation, at rest, one lattice step of
    n_sub sub-steps under a constant lab-frame torque.  After the first
    sub-step: w = (R I R^T)^-1 T dt exactly; the control points have turned
    about w by |w| dt.  A torque taken into the body frame with R instead of
    R^T, or the spin increment applied on the wrong side of the quaternion,
    fails this."""
    off, k = workloads.random_body(np.random.Generator(np.random.PCG64(17)), 7, 5.0)
    q0 = np.array([0.8, 0.3, -0.4, 0.33])
    q0 /= np.linalg.norm(q0)
    p = workloads.Particle(cp_xyz=off, cp_k=k, x=np.array([20.0, 20.0, 20.0]), quat=q0, density=2.0)
    cfg = workloads.Config(nx=40, ny=40, nz=40, periodic=7, tau=0.8, n_sub=1, particles=[p])
    o = oracle.Oracle(cfg)
    P = o.particle(0)
    R = quat_rot(P["quat"])
    I_lab = R @ P["I"] @ R.T
    T = np.array([3e-3, -1e-3, 2e-3])
    lab0, _ = o.cps(0)
    o.rigid_body_step(0, np.zeros(3), T)
    Q = o.particle(0)
    w = np.linalg.solve(I_lab, T)
    assert np.allclose(Q["omega"], w, rtol=1e-12, atol=1e-18)
    lab1, _ = o.cps(0)
    assert np.allclose(Q["x"], P["x"], atol=1e-14)
    expect = P["x"] + rodrigues(w, lab0 - P["x"])
    assert np.abs(lab1 - expect).max() < 1e-12
    # n_sub sub-steps of 1/n_sub under the same torque end at the same spin
    # up to the gyroscopic term and the turn of the body within the step,
    # both second order in the (small) spin
    cfg.n_sub = n_sub
    o2 = oracle.Oracle(cfg)
    o2.rigid_body_step(0, np.zeros(3), T)
    assert np.linalg.norm(o2.particle(0)["omega"] - w) < 1e-5 * np.linalg.norm(w)
