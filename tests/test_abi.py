"""The C ABI without a GPU: the library loads, exports every function that
include/*.h declares, and the host-only calls (lbm_arena_bytes, the
Metaball-Imaging workspace sizes and argument checks) validate their inputs
with the documented status codes."""
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:lbm_status|void|size_t|int32_t|const char\s*\*)\s*\**\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def mdl():
    import paper_2209_10411_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2209_10411_amd import build
        build.build()
    return m


def test_header_lists_the_hot_path_calls():
    names = header_functions()
    for n in ["lbm_init", "metaball_flag", "lbm_step", "particle_forces", "refill"]:
        assert n in names


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library the binding raises at its first call: a
    simulation or an ensemble is never set up on anything else."""
    import paper_2209_10411_amd as m
    monkeypatch.setattr(m, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(m, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        m.lib()
    with pytest.raises(RuntimeError, match="missing"):
        m.Simulation(workloads.config1(), device="cpu")
    with pytest.raises(RuntimeError, match="missing"):
        m.Ensemble([workloads.config1()], device="cpu")


def test_library_exports_every_declared_symbol(mdl):
    L = mdl.lib()
    for n in header_functions():
        assert hasattr(L, n), n
    assert sorted(mdl.EXPORTS) == header_functions()


def test_arena_bytes_counts_populations(mdl):
    cfg = workloads.config1()
    b32 = mdl.arena_bytes(cfg)
    cfg.storage = workloads.STORE_F16
    b16 = mdl.arena_bytes(cfg)
    N = 64 ** 3
    assert b32 >= 2 * 19 * 4 * N
    assert b32 - b16 >= 2 * 19 * 2 * N - 1024


@pytest.mark.parametrize("mutate,code", [
    (lambda c: setattr(c, "tau", 0.5), -1),
    (lambda c: setattr(c, "nx", 2), -1),
    (lambda c: setattr(c, "storage", 7), -1),
    (lambda c: setattr(c, "n_sub", 0), -1),
    (lambda c: setattr(c, "g_fluid", np.array([np.nan, 0, 0])), -1),
    (lambda c: c.particles[0].__setattr__("cp_k", np.array([-1.0])), -1),
    (lambda c: (c.particles[0].__setattr__("cp_xyz", np.arange(63.0).reshape(21, 3) / 10),
                c.particles[0].__setattr__("cp_k", np.ones(21))), -1),
    (lambda c: c.particles[0].__setattr__("density", 0.0), -1),
])
def test_arena_bytes_rejects_bad_input(mdl, mutate, code):
    cfg = workloads.config1()
    mutate(cfg)
    with pytest.raises(mdl.LbmError) as e:
        mdl.arena_bytes(cfg)
    assert e.value.status == code
    assert mdl.lib().lbm_last_error()


def test_particle_crossing_a_wall_is_rejected(mdl):
    cfg = workloads.config2(scale=0.25)
    cfg.particles[0].x = np.array([3.0, 16.0, 50.0])
    with pytest.raises(mdl.LbmError) as e:
        mdl.arena_bytes(cfg)
    assert "wall" in str(e.value)


def _batch_args(mdl, cfgs):
    import ctypes as C
    n = len(cfgs)
    cc = (mdl.lbm_config * n)(*[mdl.make_config(c) for c in cfgs])
    parts, keep = mdl.make_particles([p for c in cfgs for p in c.particles])
    npa = (C.c_int32 * n)(*[len(c.particles) for c in cfgs])
    return n, cc, npa, parts, keep


def test_batch_arena_bytes_sums_the_systems(mdl):
    import ctypes as C
    cfgs = workloads.mini_ensemble(3)
    n, cc, npa, parts, keep = _batch_args(mdl, cfgs)
    b = C.c_size_t(0)
    assert mdl.lib().lbm_batch_arena_bytes(n, cc, npa, parts, C.byref(b)) == 0
    assert b.value >= sum(mdl.arena_bytes(c) for c in cfgs)


def test_batch_rejects_mixed_storage_and_bad_cases(mdl):
    import ctypes as C
    cfgs = workloads.mini_ensemble(2)
    cfgs[1].storage = workloads.STORE_F16
    n, cc, npa, parts, keep = _batch_args(mdl, cfgs)
    b = C.c_size_t(0)
    assert mdl.lib().lbm_batch_arena_bytes(n, cc, npa, parts, C.byref(b)) == -1
    assert b"storage" in mdl.lib().lbm_last_error()
    cfgs = workloads.mini_ensemble(2)
    cfgs[1].tau = 0.5
    n, cc, npa, parts, keep = _batch_args(mdl, cfgs)
    assert mdl.lib().lbm_batch_arena_bytes(n, cc, npa, parts, C.byref(b)) == -1
    assert b"case 1" in mdl.lib().lbm_last_error()
    assert mdl.lib().lbm_batch_arena_bytes(0, cc, npa, parts, C.byref(b)) == -1


def test_mlp_sizes_match_the_oracle(mdl):
    from oracle import mlp
    assert mdl.lib().mlp_param_count() == mlp.P == 10052
    assert mdl.lib().mlp_weights_bytes() >= 4 * 3 * mlp.P + 2 * mlp.P


@pytest.mark.parametrize("hp", ['{"batch": 0}', '{"batch": 5000}', '{"lr": -1}', '{"beta1": 1.0}',
                                '{"precision": 2}', '{"eps": 0}'])
def test_mlp_train_rejects_bad_hyperparameters(mdl, hp):
    """Rejected before any device access (the pointers are never used)."""
    import ctypes as C
    dummy = C.c_void_p(256)
    rc = mdl.lib().mlp_train(dummy, dummy, 10, hp.encode(), dummy, None)
    assert rc == -1
    assert b"hyper-parameters" in mdl.lib().lbm_last_error()


def test_mlp_grad_rejects_oversized_batches(mdl):
    import ctypes as C
    dummy = C.c_void_p(256)
    assert mdl.lib().mlp_grad(dummy, dummy, dummy, 5000, 0, None, None, None) == -1
    assert mdl.lib().mlp_grad(dummy, dummy, dummy, 10, 3, None, None, None) == -1


def test_mifit_sizes_and_argument_checks(mdl):
    L = mdl.lib()
    assert L.mi_fitness_work_bytes(2048, 10) == 0          # one chunk: no workspace
    assert L.mi_fitness_work_bytes(2049, 10) == 10 * 2 * 8  # two chunks per individual
    assert L.mi_ga_work_bytes(100, 1, 4) == 0                # N_I >= 2
    assert L.mi_ga_work_bytes(100, 8, 4) > 2 * 3 * 8 * 4 * 4 * 8
    import ctypes as C
    nul = C.c_void_p(0)
    # NULL pointers and sizes out of range are refused before any launch
    assert L.mi_fitness(nul, 10, nul, 4, 4, nul, nul, 0, nul) == -1
    assert L.mi_ga(nul, 10, 4, 4, 1, 0.6, 0.5, 0.1, 0.1, nul, nul, nul, nul, nul, nul, 0, nul) == -1
    assert L.mi_gs(nul, nul, nul, nul, 1, 4, 1, 1e-3, nul, nul, nul) == -1
