"""CPU FP64 oracle of the metaball-coupled lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does,
and the two share no code.  The arithmetic lives in ``oracle.c`` (plain C,
FP64, plain loops); this file only builds it with gcc and marshals arrays.

Every function of ``oracle.c`` cites the paper section or equation it
follows.  Pins that tie it to the paper and to mathematics (not to itself)
are in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-std=c11",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint, C.c_double, C.c_double,
                                 _dp, _dp, C.c_int, C.c_int, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_add_particle.restype = C.c_int
        L.orc_add_particle.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp,
                                       C.c_double, C.c_int, C.c_double]
        L.orc_init.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        for name in ("orc_n_nodes", "orc_n_links", "orc_n_refilled"):
            getattr(L, name).restype = C.c_long
            getattr(L, name).argtypes = [C.c_void_p]
        L.orc_n_particles.argtypes = [C.c_void_p]
        L.orc_get_gfluid.argtypes = [C.c_void_p, _dp]
        L.orc_get_f.argtypes = [C.c_void_p, _dp]
        L.orc_set_f.argtypes = [C.c_void_p, _dp]
        L.orc_get_fpost.argtypes = [C.c_void_p, _dp]
        L.orc_get_macros.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_get_owner.argtypes = [C.c_void_p, _i32p]
        L.orc_get_links.argtypes = [C.c_void_p, _i64p, _i32p, _i32p, _dp]
        L.orc_get_particle.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_set_particle_state.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
        L.orc_get_cps.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_reflag.argtypes = [C.c_void_p]
        L.orc_rigid_body_step.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_link_q.restype = C.c_double
        L.orc_link_q.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_metaball_eval.restype = C.c_double
        L.orc_metaball_eval.argtypes = [C.c_int, _dp, _dp, _dp]
        L.orc_body_properties.argtypes = [C.c_int, _dp, _dp, C.c_double, _dp, _dp, _dp,
                                          C.POINTER(C.c_long)]
        L.orc_feq.argtypes = [C.c_double, _dp, _dp]
        L.orc_collide_node.argtypes = [_dp, _dp, C.c_double, _dp]
        L.orc_lattice.argtypes = [_i32p, _dp, _i32p]
        L.orc_set_contact.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_set_link_c0.argtypes = [C.c_void_p, C.c_int]
        L.orc_pair_geometry.restype = C.c_int
        L.orc_pair_geometry.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_wall_geometry.restype = C.c_int
        L.orc_wall_geometry.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_dem_only.argtypes = [C.c_void_p, C.c_int]
        L.orc_n_contacts.restype = C.c_long
        L.orc_n_contacts.argtypes = [C.c_void_p]
        L.orc_n_contact_fail.restype = C.c_long
        L.orc_n_contact_fail.argtypes = [C.c_void_p]
        L.orc_threads.restype = C.c_int
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _a(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def lattice():
    """(e (19,3) int, w (19,), opposite index (19,)) as the oracle uses them."""
    e, w, op = np.zeros(57, np.int32), np.zeros(19), np.zeros(19, np.int32)
    lib().orc_lattice(e, w, op)
    return e.reshape(19, 3), w, op


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    """Number of OpenMP threads of the oracle's loops from now on."""
    lib().orc_set_threads(int(n))


def feq(rho: float, u) -> np.ndarray:
    out = np.zeros(19)
    lib().orc_feq(float(rho), _a(u, 3), out)
    return out


def collide_node(f, g, tau: float) -> np.ndarray:
    out = np.zeros(19)
    lib().orc_collide_node(_a(f, 19), _a(g, 3), float(tau), out)
    return out


def metaball_eval(cp_xyz, cp_k, x) -> float:
    cp = _a(cp_xyz)
    return lib().orc_metaball_eval(len(cp) // 3, cp, _a(cp_k), _a(x, 3))


def body_properties(cp_xyz, cp_k, h: float = 0.125):
    """Volume, centroid, inertia (per unit density) and sample count."""
    cp = _a(cp_xyz)
    V, c, I, cnt = np.zeros(1), np.zeros(3), np.zeros(9), C.c_long(0)
    rc = lib().orc_body_properties(len(cp) // 3, cp, _a(cp_k), float(h), V, c, I, C.byref(cnt))
    if rc:
        raise ValueError("empty body")
    return float(V[0]), c, I.reshape(3, 3), int(cnt.value)


class Oracle:
    """One simulation state advanced by the oracle's canonical step."""

    def __init__(self, cfg):
        L = lib()
        self.cfg = cfg
        self.N = cfg.nx * cfg.ny * cfg.nz
        self._h = L.orc_create(cfg.nx, cfg.ny, cfg.nz, cfg.periodic, cfg.tau, cfg.rho0,
                               _a(cfg.g_fluid, 3), _a(cfg.g_particle, 3), cfg.bc, cfg.n_sub,
                               cfg.counter_force)
        if not self._h:
            raise ValueError("oracle rejected the configuration")
        for p in cfg.particles:
            rc = L.orc_add_particle(self._h, p.n_cp, _a(p.cp_xyz), _a(p.cp_k), _a(p.x, 3),
                                    _a(p.quat, 4), _a(p.v, 3), _a(p.omega, 3), float(p.density),
                                    int(p.mode), float(cfg.quad_h))
            if rc < 0:
                raise ValueError("oracle rejected a particle")
        L.orc_set_contact(self._h, float(cfg.contact_rs), float(cfg.contact_kn),
                          float(cfg.contact_en), float(cfg.contact_mu))
        L.orc_init(self._h)
        if getattr(cfg, "link_c0", 0):
            L.orc_set_link_c0(self._h, 1)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    @property
    def n_links(self) -> int:
        return lib().orc_n_links(self._h)

    @property
    def n_refilled(self) -> int:
        return lib().orc_n_refilled(self._h)

    @property
    def g_fluid(self) -> np.ndarray:
        g = np.zeros(3)
        lib().orc_get_gfluid(self._h, g)
        return g

    def f(self) -> np.ndarray:
        out = np.zeros(19 * self.N)
        lib().orc_get_f(self._h, out)
        return out.reshape(19, self.N)

    def set_f(self, f):
        lib().orc_set_f(self._h, _a(f, 19 * self.N))

    def fpost(self) -> np.ndarray:
        out = np.zeros(19 * self.N)
        lib().orc_get_fpost(self._h, out)
        return out.reshape(19, self.N)

    def macros(self):
        rho, u = np.zeros(self.N), np.zeros(3 * self.N)
        lib().orc_get_macros(self._h, rho, u)
        return rho, u.reshape(self.N, 3)

    def owner(self) -> np.ndarray:
        o = np.zeros(self.N, dtype=np.int32)
        lib().orc_get_owner(self._h, o)
        return o

    def links(self):
        n = self.n_links
        node, d, o, q = (np.zeros(n, np.int64), np.zeros(n, np.int32),
                         np.zeros(n, np.int32), np.zeros(n))
        if n:
            lib().orc_get_links(self._h, node, d, o, q)
        return node, d, o, q

    def particle(self, p: int) -> dict:
        r = np.zeros(32)
        lib().orc_get_particle(self._h, p, r)
        return {"x": r[0:3], "quat": r[3:7], "v": r[7:10], "omega": r[10:13], "F": r[13:16],
                "T": r[16:19], "m": r[19], "V": r[20], "I": r[21:30].reshape(3, 3),
                "rb": r[30], "n_cp": int(r[31])}

    def set_particle_state(self, p, x, quat, v, omega):
        lib().orc_set_particle_state(self._h, p, _a(x, 3), _a(quat, 4), _a(v, 3), _a(omega, 3))

    def cps(self, p: int):
        lab, k = np.zeros(3 * 20), np.zeros(20)
        n = lib().orc_get_cps(self._h, p, lab, k)
        return lab[:3 * n].reshape(n, 3), k[:n]

    def reflag(self):
        lib().orc_reflag(self._h)

    def rigid_body_step(self, p: int, F, T):
        lib().orc_rigid_body_step(self._h, p, _a(F, 3), _a(T, 3))

    def link_q(self, p: int, x: int, y: int, z: int, i: int) -> float:
        return lib().orc_link_q(self._h, p, x, y, z, i)

    def pair_geometry(self, i: int, j: int):
        """(status, x_m, x_c0, x_c1, x_cp, n, delta) of bodies i, j."""
        xm, xc0, xc1, xcp, n, d = [np.zeros(3) for _ in range(5)] + [np.zeros(1)]
        r = lib().orc_pair_geometry(self._h, i, j, xm, xc0, xc1, xcp, n, d)
        return r, xm, xc0, xc1, xcp, n, float(d[0])

    def wall_geometry(self, p: int, axis: int, side: int):
        """(status, x_cw, x_cm, x_cp, n, delta) of body p and a walled face."""
        xcw, xcm, xcp, n, d = [np.zeros(3) for _ in range(4)] + [np.zeros(1)]
        r = lib().orc_wall_geometry(self._h, p, axis, side, xcw, xcm, xcp, n, d)
        return r, xcw, xcm, xcp, n, float(d[0])

    def dem_only(self, n: int):
        lib().orc_dem_only(self._h, int(n))

    @property
    def n_contacts(self) -> int:
        return lib().orc_n_contacts(self._h)

    @property
    def n_contact_fail(self) -> int:
        return lib().orc_n_contact_fail(self._h)
