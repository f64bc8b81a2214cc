"""Python binding of libmidelbm.so, the MI355X (gfx950) HIP implementation of
the per-step hot path of MI-DELBM (arXiv 2209.10411): metaball flagging,
D3Q19 BGK stream-collide with (interpolated) bounce-back on metaball-cut
links, momentum-exchange force and torque, FP64 rigid-body update and local
refilling.

This module only marshals arguments.  Every step of the path runs in the HIP
kernels behind the C ABI declared in include/midelbm.h; PyTorch provides the
device arena and the stream.  If the shared library is missing the import of
``lib()`` raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmidelbm.so")

LBM_STORE_F32, LBM_STORE_F16, LBM_STORE_BF16 = 0, 1, 2
LBM_BC_SBB, LBM_BC_IBB = 0, 1
LBM_STEP_FLUID_ONLY, LBM_STEP_COUPLED = 0, 1

_STATUS = {0: "LBM_OK", -1: "LBM_E_INVALID", -2: "LBM_E_NOMEM", -3: "LBM_E_HIP",
           -4: "LBM_E_DIVERGED", -5: "LBM_E_STATE"}


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class lbm_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("periodic", C.c_uint32),
                ("tau", C.c_double), ("rho0", C.c_double), ("g_fluid", C.c_double * 3),
                ("g_particle", C.c_double * 3), ("storage", C.c_int32), ("bc", C.c_int32),
                ("n_sub", C.c_int32), ("counter_force", C.c_int32), ("quad_h", C.c_double),
                ("fp16_scale", C.c_float), ("link_c0", C.c_int32),
                ("contact_rs", C.c_double), ("contact_kn", C.c_double), ("contact_en", C.c_double),
                ("contact_mu", C.c_double)]


class lbm_particle(C.Structure):
    _fields_ = [("n_cp", C.c_int32), ("mode", C.c_int32), ("cp_xyz", C.POINTER(C.c_double)),
                ("cp_k", C.POINTER(C.c_double)), ("x", C.c_double * 3), ("quat", C.c_double * 4),
                ("v", C.c_double * 3), ("omega", C.c_double * 3), ("density", C.c_double)]


class lbm_particle_state(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("quat", C.c_double * 4), ("v", C.c_double * 3),
                ("omega", C.c_double * 3), ("F", C.c_double * 3), ("T", C.c_double * 3),
                ("mass", C.c_double), ("volume", C.c_double), ("inertia", C.c_double * 9)]


class mb_shape(C.Structure):
    _fields_ = [("V", C.c_double), ("S", C.c_double), ("A_p", C.c_double), ("dims", C.c_double * 3),
                ("axes", C.c_double * 9), ("centroid", C.c_double * 3), ("d_n", C.c_double), ("d_s", C.c_double),
                ("Phi", C.c_double), ("CSF", C.c_double), ("cells_inside", C.c_int64), ("columns_hit", C.c_int64)]


EXPORTS = ["lbm_arena_bytes", "lbm_init", "metaball_flag", "lbm_step", "particle_forces", "refill",
           "lbm_get_macros", "lbm_get_populations", "lbm_set_populations", "lbm_get_flags",
           "lbm_get_links", "lbm_get_particles", "lbm_set_particles", "lbm_get_gfluid",
           "lbm_timing_enable", "lbm_timing_read", "lbm_nr_stats", "lbm_contact_stats", "lbm_contact_nr_stats",
           "lbm_sync", "lbm_save", "lbm_load", "lbm_copy_probe",
           "lbm_destroy",
           "lbm_last_error",
           "lbm_batch_arena_bytes", "lbm_batch_init", "lbm_batch_step", "lbm_batch_case", "lbm_autotune",
           "lbm_batch_tiles", "lbm_batch_destroy",
           "mlp_weights_bytes", "mlp_param_count", "mlp_init", "mlp_get_params", "mlp_collect",
           "mlp_collect_contact", "mlp_forward",
           "mlp_grad", "mlp_train", "lbm_set_warmstart", "lbm_nr_histogram",
           "mi_fitness_work_bytes", "mi_fitness", "mi_fitness_noalloc", "mi_ga_work_bytes", "mi_ga", "mi_gs",
           "mb_shape_work_bytes", "mb_shape_descriptors"]

_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python paper_2209_10411_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.lbm_arena_bytes.argtypes = [C.POINTER(lbm_config), C.c_int32, C.POINTER(lbm_particle),
                                      C.POINTER(C.c_size_t)]
        L.lbm_init.argtypes = [C.POINTER(lbm_config), C.c_int32, C.POINTER(lbm_particle), vp,
                               C.c_size_t, vp, C.POINTER(vp)]
        L.metaball_flag.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.lbm_step.argtypes = [vp, C.c_int32, C.c_int32]
        L.particle_forces.argtypes = [vp, dp, dp]
        L.refill.argtypes = [vp, C.POINTER(C.c_int64)]
        L.lbm_get_macros.argtypes = [vp, dp, dp]
        L.lbm_get_populations.argtypes = [vp, dp]
        L.lbm_set_populations.argtypes = [vp, dp, C.c_int32]
        L.lbm_get_flags.argtypes = [vp, C.POINTER(C.c_int32)]
        L.lbm_get_links.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_uint32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp]
        L.lbm_get_particles.argtypes = [vp, C.POINTER(lbm_particle_state)]
        L.lbm_set_particles.argtypes = [vp, C.POINTER(lbm_particle_state)]
        L.lbm_get_gfluid.argtypes = [vp, dp]
        L.lbm_timing_enable.argtypes = [vp, C.c_int32]
        L.lbm_timing_read.argtypes = [vp, dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.lbm_nr_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.lbm_contact_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.lbm_contact_nr_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.lbm_sync.argtypes = [vp]
        L.lbm_copy_probe.argtypes = [vp, vp, C.c_int64, C.c_int64, C.c_int32, C.c_int32, vp, dp]
        L.lbm_save.argtypes = [vp, C.c_char_p]
        L.lbm_load.argtypes = [vp, C.c_char_p]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_destroy.restype = None
        L.lbm_last_error.restype = C.c_char_p
        ip = C.POINTER(C.c_int32)
        L.lbm_batch_arena_bytes.argtypes = [C.c_int32, C.POINTER(lbm_config), ip, C.POINTER(lbm_particle),
                                            C.POINTER(C.c_size_t)]
        L.lbm_batch_init.argtypes = [C.c_int32, C.POINTER(lbm_config), ip, C.POINTER(lbm_particle), vp,
                                     C.c_size_t, vp, C.POINTER(vp)]
        L.lbm_batch_step.argtypes = [vp, C.c_int32, C.c_int32]
        L.lbm_batch_case.argtypes = [vp, C.c_int32, C.POINTER(vp)]
        L.lbm_autotune.argtypes = [vp, C.c_double, C.c_char_p]
        L.lbm_batch_tiles.argtypes = [vp, ip, ip]
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_batch_destroy.restype = None
        L.mlp_weights_bytes.argtypes = []
        L.mlp_weights_bytes.restype = C.c_size_t
        L.mlp_param_count.argtypes = []
        L.mlp_param_count.restype = C.c_int32
        fp = C.POINTER(C.c_float)
        L.mlp_init.argtypes = [vp, fp, vp]
        L.mlp_get_params.argtypes = [vp, fp, vp]
        L.mlp_collect.argtypes = [vp, C.c_int64, vp, vp, C.POINTER(C.c_int64)]
        L.mlp_collect_contact.argtypes = [vp, C.c_int64, vp, vp, C.POINTER(C.c_int64)]
        L.mlp_forward.argtypes = [vp, vp, C.c_int64, C.c_int32, vp, vp]
        L.mlp_grad.argtypes = [vp, vp, vp, C.c_int64, C.c_int32, fp, dp, vp]
        L.mlp_train.argtypes = [vp, vp, C.c_int64, C.c_char_p, vp, vp]
        L.lbm_set_warmstart.argtypes = [vp, vp]
        L.lbm_nr_histogram.argtypes = [vp, C.POINTER(C.c_int64), dp]
        L.mi_fitness_work_bytes.argtypes = [C.c_int64, C.c_int32]
        L.mi_fitness_work_bytes.restype = C.c_size_t
        L.mi_fitness.argtypes = [vp, C.c_int64, vp, C.c_int32, C.c_int32, vp, vp, C.c_size_t, vp]
        L.mi_fitness_noalloc.argtypes = [vp, C.c_int64, vp, C.c_int32, C.c_int32, vp, vp]
        L.mi_ga_work_bytes.argtypes = [C.c_int64, C.c_int32, C.c_int32]
        L.mi_ga_work_bytes.restype = C.c_size_t
        L.mi_ga.argtypes = [vp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double,
                            C.c_double, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.mi_gs.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, vp, vp, vp]
        L.mb_shape_work_bytes.argtypes = [dp, dp, C.c_int32, C.c_double]
        L.mb_shape_work_bytes.restype = C.c_size_t
        L.mb_shape_descriptors.argtypes = [dp, dp, C.c_int32, C.c_double, vp, C.c_size_t, vp, C.POINTER(mb_shape)]
        for name in EXPORTS:
            if name not in ("lbm_destroy", "lbm_last_error", "lbm_batch_destroy", "mlp_weights_bytes",
                            "mlp_param_count", "mi_fitness_work_bytes", "mi_ga_work_bytes",
                            "mb_shape_work_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise LbmError(rc, lib().lbm_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_config(cfg) -> lbm_config:
    c = lbm_config()
    c.nx, c.ny, c.nz, c.periodic = cfg.nx, cfg.ny, cfg.nz, cfg.periodic
    c.tau, c.rho0 = cfg.tau, cfg.rho0
    c.g_fluid[:] = [float(v) for v in cfg.g_fluid]
    c.g_particle[:] = [float(v) for v in cfg.g_particle]
    c.storage, c.bc, c.n_sub = int(cfg.storage), int(cfg.bc), int(cfg.n_sub)
    c.counter_force = int(cfg.counter_force)
    c.quad_h = float(cfg.quad_h)
    c.fp16_scale = float(getattr(cfg, "fp16_scale", 0.0))
    c.contact_rs = float(getattr(cfg, "contact_rs", 1.0))
    c.contact_kn = float(getattr(cfg, "contact_kn", 0.0))
    c.contact_en = float(getattr(cfg, "contact_en", 0.5))
    c.contact_mu = float(getattr(cfg, "contact_mu", 0.5))
    c.link_c0 = int(getattr(cfg, "link_c0", 0))
    return c


def make_particles(parts):
    """ctypes array of lbm_particle plus the numpy buffers it points into."""
    arr = (lbm_particle * max(len(parts), 1))()
    keep = []
    for j, p in enumerate(parts):
        cp = np.ascontiguousarray(p.cp_xyz, dtype=np.float64).reshape(-1)
        k = np.ascontiguousarray(p.cp_k, dtype=np.float64)
        keep += [cp, k]
        a = arr[j]
        a.n_cp, a.mode = int(k.size), int(p.mode)
        a.cp_xyz, a.cp_k = _dptr(cp), _dptr(k)
        a.x[:] = [float(v) for v in p.x]
        a.quat[:] = [float(v) for v in p.quat]
        a.v[:] = [float(v) for v in p.v]
        a.omega[:] = [float(v) for v in p.omega]
        a.density = float(p.density)
    return arr, keep


def arena_bytes(cfg) -> int:
    c = make_config(cfg)
    parts, keep = make_particles(cfg.particles)
    n = C.c_size_t(0)
    _check(lib().lbm_arena_bytes(C.byref(c), len(cfg.particles), parts, C.byref(n)))
    return int(n.value)


class Simulation:
    """A coupled metaball/LBM system on one GPU.  ``cfg`` is any object with
    the fields of ``workloads.Config`` (sizes, tau, rho0, forces, storage,
    boundary rule, particles)."""

    def __init__(self, cfg, device: str = "cuda:0", stream=None):
        import torch

        self.cfg = cfg
        self.N = cfg.nx * cfg.ny * cfg.nz
        self.np = len(cfg.particles)
        self.device = torch.device(device)
        L = lib()
        c = make_config(cfg)
        parts, keep = make_particles(cfg.particles)
        n = C.c_size_t(0)
        _check(L.lbm_arena_bytes(C.byref(c), self.np, parts, C.byref(n)))
        self.arena = torch.empty(int(n.value), dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = C.c_void_p()
        _check(L.lbm_init(C.byref(c), self.np, parts, C.c_void_p(self.arena.data_ptr()),
                          self.arena.numel(), C.c_void_p(self.stream.cuda_stream),
                          C.byref(self._ctx)))

    @classmethod
    def _view(cls, ctx: C.c_void_p, cfg, owner):
        """A system owned by an Ensemble (not destroyed by this object)."""
        self = cls.__new__(cls)
        self.cfg, self.N, self.np = cfg, cfg.nx * cfg.ny * cfg.nz, len(cfg.particles)
        self._ctx, self._owner = ctx, owner
        return self

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self._ctx = C.c_void_p()
            return
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().lbm_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- the five calls of the hot path
    def metaball_flag(self, counts: bool = True):
        ns, nl = C.c_int64(0), C.c_int64(0)
        if counts:
            _check(lib().metaball_flag(self._ctx, C.byref(ns), C.byref(nl)))
            return int(ns.value), int(nl.value)
        _check(lib().metaball_flag(self._ctx, None, None))
        return None

    def step(self, n: int = 1, coupled: bool = True):
        _check(lib().lbm_step(self._ctx, int(n), LBM_STEP_COUPLED if coupled else LBM_STEP_FLUID_ONLY))

    def particle_forces(self):
        F, T = np.zeros(3 * self.np), np.zeros(3 * self.np)
        _check(lib().particle_forces(self._ctx, _dptr(F), _dptr(T)))
        return F.reshape(-1, 3), T.reshape(-1, 3)

    def refill(self) -> int:
        n = C.c_int64(0)
        _check(lib().refill(self._ctx, C.byref(n)))
        return int(n.value)

    # ---- state access
    def sync(self):
        _check(lib().lbm_sync(self._ctx))

    def save(self, path: str):
        """Checkpoint of the whole state (lbm_save)."""
        _check(lib().lbm_save(self._ctx, os.fsencode(path)))

    def load(self, path: str):
        """Replaces the state with a checkpoint of the same configuration (lbm_load)."""
        _check(lib().lbm_load(self._ctx, os.fsencode(path)))

    def macros(self):
        rho, u = np.zeros(self.N), np.zeros(3 * self.N)
        _check(lib().lbm_get_macros(self._ctx, _dptr(rho), _dptr(u)))
        return rho, u.reshape(self.N, 3)

    def populations(self) -> np.ndarray:
        f = np.zeros(19 * self.N)
        _check(lib().lbm_get_populations(self._ctx, _dptr(f)))
        return f.reshape(19, self.N)

    def set_populations(self, f, post_collision: bool = False):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        if a.size != 19 * self.N:
            raise ValueError("populations must have 19*N values")
        _check(lib().lbm_set_populations(self._ctx, _dptr(a), int(bool(post_collision))))

    def owner(self) -> np.ndarray:
        o = np.zeros(self.N, dtype=np.int32)
        _check(lib().lbm_get_flags(self._ctx, o.ctypes.data_as(C.POINTER(C.c_int32))))
        return o

    def links(self):
        n = C.c_int64(0)
        _check(lib().lbm_get_links(self._ctx, C.byref(n), None, None, None, None))
        nl = int(n.value)
        node, d = np.zeros(nl, np.uint32), np.zeros(nl, np.int32)
        o, q = np.zeros(nl, np.int32), np.zeros(nl)
        if nl:
            _check(lib().lbm_get_links(self._ctx, C.byref(n),
                                       node.ctypes.data_as(C.POINTER(C.c_uint32)),
                                       d.ctypes.data_as(C.POINTER(C.c_int32)),
                                       o.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(q)))
        return node.astype(np.int64), d, o, q

    def particles(self):
        arr = (lbm_particle_state * max(self.np, 1))()
        _check(lib().lbm_get_particles(self._ctx, arr))
        out = []
        for j in range(self.np):
            s = arr[j]
            out.append({"x": np.array(s.x[:]), "quat": np.array(s.quat[:]), "v": np.array(s.v[:]),
                        "omega": np.array(s.omega[:]), "F": np.array(s.F[:]), "T": np.array(s.T[:]),
                        "m": s.mass, "V": s.volume, "I": np.array(s.inertia[:]).reshape(3, 3)})
        return out

    def set_particles(self, states):
        arr = (lbm_particle_state * max(self.np, 1))()
        for j, st in enumerate(states):
            a = arr[j]
            a.x[:] = [float(v) for v in st["x"]]
            a.quat[:] = [float(v) for v in st["quat"]]
            a.v[:] = [float(v) for v in st["v"]]
            a.omega[:] = [float(v) for v in st["omega"]]
        _check(lib().lbm_set_particles(self._ctx, arr))

    def g_fluid(self) -> np.ndarray:
        g = np.zeros(3)
        _check(lib().lbm_get_gfluid(self._ctx, _dptr(g)))
        return g

    # ---- measurement
    def nr_stats(self):
        """(link fractions solved, Newton/bisection iterations) since the last call."""
        a, b = C.c_int64(0), C.c_int64(0)
        _check(lib().lbm_nr_stats(self._ctx, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def contact_stats(self):
        """(contacts resolved, failed contact iterations) since initialisation."""
        a, b = C.c_int64(0), C.c_int64(0)
        _check(lib().lbm_contact_stats(self._ctx, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def contact_nr_stats(self):
        """(pair stationary-point solves, their Newton evaluations) since the last call."""
        a, b = C.c_int64(0), C.c_int64(0)
        _check(lib().lbm_contact_nr_stats(self._ctx, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def nr_histogram(self):
        """(histogram of Newton evaluations per link [65], largest final |C - 1|) since the last call."""
        h = np.zeros(65, dtype=np.int64)
        r = C.c_double(0)
        _check(lib().lbm_nr_histogram(self._ctx, h.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(r)))
        return h, float(r.value)

    def set_warmstart(self, mlp):
        """Warm-start the link fractions with an ``Mlp`` (None: plain Newton)."""
        self._warm = mlp
        _check(lib().lbm_set_warmstart(self._ctx, C.c_void_p(mlp.blob.data_ptr()) if mlp is not None else None))

    def timing(self, on: bool = True, every: int = 1):
        """Time the stream-collide of every `every`-th step with HIP events."""
        _check(lib().lbm_timing_enable(self._ctx, max(1, int(every)) if on else 0))

    def timing_read(self):
        ms, n, nodes = C.c_double(0), C.c_int64(0), C.c_int64(0)
        _check(lib().lbm_timing_read(self._ctx, C.byref(ms), C.byref(n), C.byref(nodes)))
        return float(ms.value), int(n.value), int(nodes.value)


class Ensemble:
    """Independent systems (a list of ``workloads.Config``) stepped together:
    one batched stream-collide launch over all of them, one batched launch
    per kind of boundary kernel, six-step HIP graph replays
    (include/midelbm.h, ensemble)."""

    def __init__(self, cfgs, device: str = "cuda:0", stream=None):
        import torch

        self.cfgs = list(cfgs)
        n = len(self.cfgs)
        L = lib()
        self._c = (lbm_config * n)(*[make_config(c) for c in self.cfgs])
        allp = [p for c in self.cfgs for p in c.particles]
        self._parts, self._keep = make_particles(allp)
        self._np = (C.c_int32 * n)(*[len(c.particles) for c in self.cfgs])
        nb = C.c_size_t(0)
        _check(L.lbm_batch_arena_bytes(n, self._c, self._np, self._parts, C.byref(nb)))
        self.device = torch.device(device)
        self.arena = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._b = C.c_void_p()
        _check(L.lbm_batch_init(n, self._c, self._np, self._parts, C.c_void_p(self.arena.data_ptr()),
                                self.arena.numel(), C.c_void_p(self.stream.cuda_stream), C.byref(self._b)))
        self.cases = []
        for i, cfg in enumerate(self.cfgs):
            ctx = C.c_void_p()
            _check(L.lbm_batch_case(self._b, i, C.byref(ctx)))
            self.cases.append(Simulation._view(ctx, cfg, self))

    def step(self, n: int = 1, graph: bool = True):
        _check(lib().lbm_batch_step(self._b, int(n), int(bool(graph))))

    def autotune(self, budget_ms: float = 2000.0, cache: str | None = None):
        _check(lib().lbm_autotune(self._b, float(budget_ms), cache.encode() if cache else None))
        return self.tiles()

    def tiles(self):
        """(per-system tile width log2, waves per block)."""
        t = (C.c_int32 * len(self.cfgs))()
        w = C.c_int32(0)
        _check(lib().lbm_batch_tiles(self._b, t, C.byref(w)))
        return list(t), int(w.value)

    def sync(self):
        for c in self.cases:
            c.sync()

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            for c in self.cases:
                c._ctx = C.c_void_p()
            lib().lbm_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """Warm-start MLP parameters, Adam state and workspace in one device blob
    (include/midelbm.h, warm start)."""

    N_IN, N_OUT = 87, 4

    def __init__(self, params, device: str = "cuda:0", stream=None):
        import torch

        L = lib()
        self.P = int(L.mlp_param_count())
        self.device = torch.device(device)
        self.blob = torch.empty(int(L.mlp_weights_bytes()), dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.load(params)

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def load(self, params):
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != self.P:
            raise ValueError(f"expected {self.P} parameters")
        _check(lib().mlp_init(C.c_void_p(self.blob.data_ptr()), a.ctypes.data_as(C.POINTER(C.c_float)), self._s()))

    def params(self) -> np.ndarray:
        a = np.zeros(self.P, dtype=np.float32)
        _check(lib().mlp_get_params(C.c_void_p(self.blob.data_ptr()), a.ctypes.data_as(C.POINTER(C.c_float)),
                                    self._s()))
        return a

    def forward(self, feat, precision: int = 0):
        """feat: device tensor [n][87] (float16 for precision 0 and 2, float32
        for 1); precision 2 runs the hidden layers on the matrix cores."""
        import torch
        n = feat.shape[0]
        out = torch.empty((n, self.N_OUT), dtype=torch.float32, device=self.device)
        _check(lib().mlp_forward(C.c_void_p(self.blob.data_ptr()), C.c_void_p(feat.data_ptr()), n, int(precision),
                                 C.c_void_p(out.data_ptr()), self._s()))
        return out

    def grad(self, feat, target, precision: int = 0):
        g = np.zeros(self.P, dtype=np.float32)
        loss = C.c_double(0)
        _check(lib().mlp_grad(C.c_void_p(self.blob.data_ptr()), C.c_void_p(feat.data_ptr()),
                              C.c_void_p(target.data_ptr()), feat.shape[0], int(precision),
                              g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss), self._s()))
        return g, float(loss.value)

    def train(self, feat, target, **hp):
        import json
        _check(lib().mlp_train(C.c_void_p(feat.data_ptr()), C.c_void_p(target.data_ptr()), feat.shape[0],
                               json.dumps(hp).encode(), C.c_void_p(self.blob.data_ptr()), self._s()))


def mlp_collect_contact(sim, n_max: int | None = None):
    """Closest-point training samples (features float16 [n][87], targets
    float32 [n][4]) from the last contact sub-step of a Simulation."""
    import torch
    L = lib()
    if n_max is None:
        n_max = max(1, sim.np * (sim.np - 1) // 2)
    feat = torch.empty((n_max, Mlp.N_IN), dtype=torch.float16, device="cuda:0")
    target = torch.empty((n_max, Mlp.N_OUT), dtype=torch.float32, device="cuda:0")
    n = C.c_int64(0)
    _check(L.mlp_collect_contact(sim._ctx, int(n_max), C.c_void_p(feat.data_ptr()),
                                 C.c_void_p(target.data_ptr()), C.byref(n)))
    return feat[:n.value], target[:n.value]


def mlp_collect(sim, n_max: int | None = None):
    """Training samples (features float16 [n][87], targets float32 [n][4])
    from the current cut links of a Simulation."""
    import torch
    L = lib()
    if n_max is None:
        n_max = len(sim.links()[0])
    feat = torch.empty((n_max, Mlp.N_IN), dtype=torch.float16, device="cuda:0")
    target = torch.empty((n_max, Mlp.N_OUT), dtype=torch.float32, device="cuda:0")
    n = C.c_int64(0)
    _check(L.mlp_collect(sim._ctx, int(n_max), C.c_void_p(feat.data_ptr()), C.c_void_p(target.data_ptr()),
                         C.byref(n)))
    return feat[:n.value], target[:n.value]


def copy_probe(n: int, elem_bytes: int = 4, reps: int = 20, device: str = "cuda:0") -> float:
    """Mean milliseconds of one streaming copy of 19 arrays of n elements
    (read + non-temporal write, lbm_copy_probe) on the current stream of
    ``device``; buffers are allocated here and freed on return."""
    import torch

    stride = (n + 1023) // 1024 * 1024  # the population layout's padded node count
    dev = torch.device(device)
    src = torch.zeros(19 * stride * elem_bytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    ms = C.c_double(0.0)
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev)
        rc = lib().lbm_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), int(n), int(stride),
                                  int(elem_bytes), int(reps), C.c_void_p(stream.cuda_stream), C.byref(ms))
    if rc != 0:
        raise LbmError(rc, "lbm_copy_probe failed")
    del src, dst
    return float(ms.value)


# ---- Metaball-Imaging fit (include/mifit.h): numpy in, numpy out; device
# buffers are torch tensors allocated here for the call
def _dev(a, dtype, device):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(device)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream(device):
    import torch
    return C.c_void_p(torch.cuda.current_stream(torch.device(device)).cuda_stream)


def mi_fitness(hull, pop, device: str = "cuda:0", work=None):
    """F [P] of the individuals pop [P][n][4] over the hull [m][3] (mi_fitness)."""
    import torch
    hull = np.asarray(hull, dtype=np.float64).reshape(-1, 3)
    pop = np.asarray(pop, dtype=np.float64)
    P, n = pop.shape[0], pop.shape[1]
    h, p = _dev(hull, torch.float64, device), _dev(pop, torch.float64, device)
    F = torch.empty(P, dtype=torch.float64, device=device)
    wb = lib().mi_fitness_work_bytes(hull.shape[0], P)
    w = torch.empty(max(int(wb), 1), dtype=torch.uint8, device=device)
    _check(lib().mi_fitness(_ptr(h), hull.shape[0], _ptr(p), P, n, _ptr(F), _ptr(w), int(wb), _stream(device)))
    torch.cuda.synchronize(device)
    return F.cpu().numpy()


def mi_ga(hull, pop0, E, C_m, C_c, sigma_x, sigma_k, U, Z, PERM, device: str = "cuda:0"):
    """Final population (fittest first) and fitness of Alg. GA (mi_ga)."""
    import torch
    hull = np.asarray(hull, dtype=np.float64).reshape(-1, 3)
    pop0 = np.asarray(pop0, dtype=np.float64)
    N, n = pop0.shape[0], pop0.shape[1]
    h, p = _dev(hull, torch.float64, device), _dev(pop0, torch.float64, device)
    u, z = _dev(U[:E], torch.float64, device), _dev(Z[:E], torch.float64, device)
    pm = _dev(PERM[:E], torch.int32, device)
    F = torch.empty(N, dtype=torch.float64, device=device)
    wb = int(lib().mi_ga_work_bytes(hull.shape[0], N, n))
    w = torch.empty(max(wb, 1), dtype=torch.uint8, device=device)
    _check(lib().mi_ga(_ptr(h), hull.shape[0], N, n, int(E), float(C_m), float(C_c), float(sigma_x),
                       float(sigma_k), _ptr(u), _ptr(z), _ptr(pm), _ptr(p), _ptr(F), _ptr(w), wb,
                       _stream(device)))
    return p.cpu().numpy(), F.cpu().numpy()


def mi_gs(hulls, planes, M0, E, eta, device: str = "cuda:0"):
    """Alg. GS for a batch: hulls and planes are lists (one per model), M0
    [B][n][4]; returns (M [B][n][4], loss [B][3])."""
    import torch
    M0 = np.asarray(M0, dtype=np.float64)
    B, n = M0.shape[0], M0.shape[1]
    ho = np.concatenate([[0], np.cumsum([len(h) for h in hulls])]).astype(np.int64)
    po = np.concatenate([[0], np.cumsum([len(q) for q in planes])]).astype(np.int64)
    H = _dev(np.concatenate([np.asarray(h, dtype=np.float64).reshape(-1, 3) for h in hulls]), torch.float64, device)
    Pl = _dev(np.concatenate([np.asarray(q, dtype=np.float64).reshape(-1, 4) for q in planes]), torch.float64, device)
    dho, dpo = _dev(ho, torch.int64, device), _dev(po, torch.int64, device)
    M = _dev(M0, torch.float64, device)
    loss = torch.empty(B * 3, dtype=torch.float64, device=device)
    _check(lib().mi_gs(_ptr(H), _ptr(dho), _ptr(Pl), _ptr(dpo), B, n, int(E), float(eta), _ptr(M), _ptr(loss),
                       _stream(device)))
    torch.cuda.synchronize(device)
    return M.cpu().numpy(), loss.cpu().numpy().reshape(B, 3)


def shape_descriptors(cp, k, h: float = 0.25, device: str = "cuda:0") -> dict:
    """Sphericity, d_n, d_s, CSF and the quantities behind them for the
    metaball (cp [n][3], k [n]) on a grid of step h (mb_shape_descriptors)."""
    import torch
    cp = np.ascontiguousarray(cp, dtype=np.float64).reshape(-1)
    k = np.ascontiguousarray(k, dtype=np.float64).reshape(-1)
    wb = int(lib().mb_shape_work_bytes(_dptr(cp), _dptr(k), k.size, float(h)))
    if wb == 0:
        raise LbmError(-1, "mb_shape_work_bytes: invalid body or grid")
    w = torch.empty(wb, dtype=torch.uint8, device=device)
    out = mb_shape()
    _check(lib().mb_shape_descriptors(_dptr(cp), _dptr(k), k.size, float(h), _ptr(w), wb, _stream(device),
                                      C.byref(out)))
    return {"V": out.V, "S": out.S, "A_p": out.A_p, "dims": np.array(out.dims[:]),
            "axes": np.array(out.axes[:]).reshape(3, 3).T, "centroid": np.array(out.centroid[:]),
            "d_n": out.d_n, "d_s": out.d_s, "Phi": out.Phi, "CSF": out.CSF,
            "cells_inside": int(out.cells_inside), "columns_hit": int(out.columns_hit)}
