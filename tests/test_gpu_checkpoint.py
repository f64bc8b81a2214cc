"""Checkpoint/resume and the fluid divergence sentinel through the C ABI.

- lbm_save after n steps, lbm_load into a fresh context of the same
  configuration, n more steps: populations, flags, cut links with q and the
  particle states are bitwise those of 2n uninterrupted steps (FP32 and FP16
  storage, a settling body that covers and uncovers nodes; two bodies with
  contact, whose tangential springs live in the state).
- A checkpoint of another configuration is refused and leaves the context
  as it was.
- A fluid node set to |u| > 0.3, or to a population that overflows FP32,
  makes the next synchronising call report LBM_E_DIVERGED; a healthy run
  reports nothing.
"""
import os

import numpy as np
import pytest

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


def _state(sim):
    return (sim.populations(), sim.owner(), sim.links(), sim.particles())


def _assert_same(a, b):
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    for x, y in zip(a[2], b[2]):
        assert np.array_equal(x, y)
    for p, q in zip(a[3], b[3]):
        for k in ("x", "quat", "v", "omega", "F", "T"):
            assert np.array_equal(p[k], q[k]), k


@pytest.mark.parametrize("case", ["settle-f32", "settle-f16", "contact-pair"])
def test_save_load_resumes_bitwise(mdl, tmp_path, case):
    if case.startswith("settle"):
        cfg = workloads.small_settling(n=32, nz=56, R=5.0, g=5e-4)
        if case.endswith("f16"):
            cfg.storage = workloads.STORE_F16
        n = 25
    else:
        cfg = workloads.contact_pair()
        n = 30
    print(f"checkpoint case {case}", flush=True)
    ref = mdl.Simulation(cfg)
    ref.step(2 * n)
    want = _state(ref)
    ref.close()
    a = mdl.Simulation(cfg)
    a.step(n)
    path = str(tmp_path / f"{case}.ckpt")
    a.save(path)
    a.step(n)
    _assert_same(_state(a), want)  # saving does not disturb the run
    a.close()
    b = mdl.Simulation(cfg)
    b.step(3)  # some other state first: the load replaces all of it
    b.load(path)
    b.step(n)
    _assert_same(_state(b), want)
    b.close()
    assert os.path.getsize(path) > 19 * cfg.n_nodes * (4 if cfg.storage == 0 else 2)


def test_load_refuses_other_configuration(mdl, tmp_path):
    cfg = workloads.small_settling(n=32, nz=56, R=5.0, g=5e-4)
    a = mdl.Simulation(cfg)
    a.step(5)
    path = str(tmp_path / "a.ckpt")
    a.save(path)
    other = cfg.copy()
    other.tau = 0.75
    b = mdl.Simulation(other)
    b.step(2)
    before = b.populations()
    with pytest.raises(mdl.LbmError) as e:
        b.load(path)
    assert e.value.status == -5  # LBM_E_STATE
    assert np.array_equal(b.populations(), before)
    with pytest.raises(mdl.LbmError) as e:
        b.load(str(tmp_path / "missing.ckpt"))
    assert e.value.status == -1


@pytest.mark.parametrize("storage", [workloads.STORE_F32, workloads.STORE_F16, workloads.STORE_BF16])
@pytest.mark.parametrize("kind", ["fast", "overflow"])
def test_divergence_sentinel(mdl, storage, kind):
    """A periodic box without bodies (every node takes the plain
    stream-collide).  'fast': the 3 x 3 x 3 block about one node is set to
    the equilibrium at |u| = 0.4, so that the node pulls every population of
    that flow; 'overflow': one population of 1e36 (finite in FP64; infinite
    once stored in FP16, a velocity near 1 in FP32 and BF16 at the node it
    streams to)."""
    cfg = workloads.Config(nx=32, ny=24, nz=20, periodic=7, tau=0.8, storage=storage)
    sim = mdl.Simulation(cfg)
    sim.step(3)
    sim.sync()  # healthy: nothing reported
    f = sim.populations()
    x, y, z = 5, 7, 9
    if kind == "fast":
        import oracle
        fe = oracle.feq(1.0, [0.4, 0.0, 0.0])
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    f[:, (x + dx) + 32 * ((y + dy) + 24 * (z + dz))] = fe
    else:
        f[1, x + 32 * (y + 24 * z)] = 1e36
    sim.set_populations(f, post_collision=True)
    sim.step(2)
    with pytest.raises(mdl.LbmError) as e:
        sim.sync()
    assert e.value.status == -4  # LBM_E_DIVERGED
    assert "fluid" in str(e.value)
