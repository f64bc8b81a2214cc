"""Writes the stored oracle results that the long-run GPU parity tests read.

Every value in the files written here comes from the FP64 CPU oracle
(``oracle/``) run on the seeded inputs of ``workloads/``; nothing is taken
from the HIP library.  Run from the repository root:

    python tests/golden/make_golden.py c2     # settling body, 128x128x384, 2000 steps
    python tests/golden/make_golden.py c3     # two bodies, 160x160x640, 5000 steps

c2_trajectory.npz: particle state every 10 steps of the single settling body
(8 control points, R = 10, density ratio 1.5, walls, tau = 0.6, gravity 2e-5;
moving interpolated bounce-back with local refilling; paper sec. 2.3.2).

c3_trajectory.npz: both bodies' states every 25 steps of the two-body case
(6 and 12 control points stacked on the axis, density ratio 1.2, contact on;
paper sec. 2.3.1 and 2.3.2), plus density and velocity at step 200 on a
fixed node sample: every node of the 25^3 cube about each body's centroid
and 8192 nodes drawn uniformly (seed 9).

Row layout of 'state' [samples][bodies][19]: x (centroid, 3), quat (w, x,
y, z), v (3), omega (3), F (3), T (3).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def _state(o, n_p):
    out = np.zeros((n_p, 19))
    for j in range(n_p):
        p = o.particle(j)
        out[j] = np.concatenate([p["x"], p["quat"], p["v"], p["omega"], p["F"], p["T"]])
    return out


def _cube_sample(cfg, centre, half):
    c = np.floor(centre).astype(int)
    r = np.arange(-half, half + 1)
    xs = np.clip(c[0] + r, 0, cfg.nx - 1)
    ys = np.clip(c[1] + r, 0, cfg.ny - 1)
    zs = np.clip(c[2] + r, 0, cfg.nz - 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return (X + cfg.nx * (Y + cfg.ny * Z)).reshape(-1)


def run(cfg, steps, every, field_step=None, path=None):
    o = oracle.Oracle(cfg)
    n_p = len(cfg.particles)
    rows, at = [_state(o, n_p)], [0]
    extra = {}
    t0 = time.time()
    for s in range(1, steps + 1):
        o.step(1)
        if s % every == 0:
            rows.append(_state(o, n_p))
            at.append(s)
        if field_step is not None and s == field_step:
            nodes = [_cube_sample(cfg, o.particle(j)["x"], 12) for j in range(n_p)]
            rng = np.random.Generator(np.random.PCG64(9))
            nodes.append(rng.integers(0, cfg.n_nodes, size=8192))
            sample = np.unique(np.concatenate(nodes))
            rho, u = o.macros()
            extra = {"field_step": np.array(field_step), "field_nodes": sample.astype(np.int64),
                     "field_rho": rho[sample], "field_u": u[sample], "field_umax":
                     np.array(np.sqrt((u * u).sum(1))[o.owner() < 0].max()),
                     "field_owner": o.owner()[sample]}
        if s % 100 == 0:
            print(f"{cfg.name}: step {s}/{steps}  {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(path, steps=np.array(at), state=np.array(rows), threads=np.array(oracle.threads()),
                        **extra)
    print("wrote", path, flush=True)


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "c2"
    if which == "c2":
        cfg = workloads.config2()
        run(cfg, 2000, 10, path=os.path.join(HERE, "c2_trajectory.npz"))
    elif which == "c3":
        cfg = workloads.config3(storage=workloads.STORE_F32)
        run(cfg, 5000, 25, field_step=200, path=os.path.join(HERE, "c3_trajectory.npz"))
    else:
        raise SystemExit("usage: make_golden.py c2|c3")


if __name__ == "__main__":
    main()
