"""Benchmark of the coupled metaball / lattice Boltzmann step on one MI355X.

Workload: the single settling particle case -- 128 x 128 x 384 lattice with
no-slip walls, D3Q19 BGK tau = 0.6, one free metaball of 8 control points
(R = 10, density ratio 1.5, gravity 2e-5), interpolated bounce-back, local
refilling; synthetic inputs from workloads.config2().  One step is one full
coupled step (cut-link bounce-back and momentum exchange, rigid body,
flagging, stream-collide with refill, cut-link rebuild).

Prints one JSON line: MLUPS over all lattice nodes with FP32 storage (the
headline), the same with FP16 storage, the roofline of the dominant kernel
(the stream-collide, timed with HIP events on the library's stream), the
64-case ensemble (batched, graph-replayed) beside the same systems stepped
one by one, the link-fraction warm start (MLP trained on the method's own
Newton solutions) against plain Newton on the 200-body suspension, and the
CPU oracle timed on a bounded sample of the headline workload.
"""
import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# the stream-collide kernel's source: its code and the data layout it reads
KERNEL_SRC = [os.path.join(ROOT, "paper_2209_10411_amd", "csrc", f) for f in ("stream_collide.h", "device.h")]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_bulk_settling_128x128x384_pmc.txt")
PMC_PAIR_SUMMARY = os.path.join(ROOT, "profiles", "k_bulk_pair_160x160x640_pmc.txt")
PMC_ENS_SUMMARY = os.path.join(ROOT, "profiles", "k_bulk_batch_ensemble_64_systems_pmc.txt")


def bytes_per_node(storage: int) -> int:
    return 19 * 2 * (4 if storage == 0 else 2)


TIMING_EVERY = 8


def run_gpu(cfg, steps, warmup, reps=1):
    """Warm-up, then `reps` timed regions of exactly `steps` coupled steps, each
    bracketed by synchronisations; returns the per-region wall times and the
    stream-collide kernel's event-timed total over all regions."""
    import torch

    import paper_2209_10411_amd as mdl

    sim = mdl.Simulation(cfg, device="cuda:0")
    sim.step(warmup)
    sim.sync()
    # the stream-collide of every 8th step is timed (events on a launch add
    # about 4.5 us to its step; a sample of 1 in 8 keeps the others free)
    sim.timing(True, every=TIMING_EVERY)
    sim.timing_read()  # reset
    dts, k_ms, k_n, k_nodes = [], 0.0, 0, 0
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        torch.cuda.synchronize()
        dts.append(time.perf_counter() - t0)
        ms, n, k_nodes = sim.timing_read()  # between regions (the event ring holds 4096 launches)
        k_ms += ms
        k_n += n
    x = sim.particles()[0]["x"]
    nr = sim.nr_stats()
    sim.close()
    return dts, k_ms, k_n, k_nodes, x, nr


def median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def run_ensemble(n_cases, steps, warmup, tune_cache=None):
    """The 64-case settling ensemble (random sizes 64..128 x 64..128 x 64..256,
    tau, density ratio, 4..16 control points; walls; FP32): autotuned tiles,
    batched launches with six-step graph replays, against the same systems
    stepped one after another with lbm_step.  tune_cache: a file of the
    autotuner's choices, read if it holds them for these systems, else
    written (so that profiler passes see the same launch shapes)."""
    import torch

    import paper_2209_10411_amd as mdl
    import workloads

    cfgs = workloads.config4(n_cases)
    nodes = sum(c.n_nodes for c in cfgs)
    ens = mdl.Ensemble(cfgs, device="cuda:0")
    t0 = time.perf_counter()
    tiles, bw = ens.autotune(budget_ms=5000.0, cache=tune_cache)
    t_tune = time.perf_counter() - t0
    ens.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same systems, one lbm_step call each (two streams per system, no batching)
    t0 = time.perf_counter()
    for sim in ens.cases:
        sim.step(steps)
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    hist = {f"{64 >> (6 - t)}x{64 >> t}": tiles.count(t) for t in (6, 5, 4)}
    hist["64 in lattice order"] = tiles.count(7)
    # algorithmic bytes of the batched stream-collide: 152 B per node it
    # updates (all but solid, boundary and uncovered ones) + 1 skip byte per node
    updated = sum(sim.timing_read()[2] for sim in ens.cases)
    alg = 152 * updated + nodes
    # the counter summary holds for the launch shape it was taken with
    tiles_key = hashlib.sha256(json.dumps([tiles, bw]).encode()).hexdigest()[:16]
    vals = profile_values(PMC_ENS_SUMMARY)
    traffic = float(vals["hbm_bytes_per_launch"]) if vals and vals.get("tiles_key") == tiles_key else None
    ens.close()
    return {"workload": f"{n_cases}-case settling ensemble, walls, FP32, 64..128 x 64..128 x 64..256, "
                        "tau U[0.55,1], density ratio U[1.1,2.5], 4..16 cp",
            "cases": n_cases, "nodes": nodes, "steps": steps,
            "value": round(nodes * steps / dt / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(dt * 1e3 / steps, 4),
            "unbatched_value": round(nodes * steps / dt_seq / 1e6, 1),
            "unbatched_ms_per_step": round(dt_seq * 1e3 / steps, 4),
            "tiles": hist, "waves_per_block": bw, "autotune_s": round(t_tune, 2),
            "algorithmic_bytes_per_step": alg,
            "traffic": traffic, "traffic_over_algorithmic": round(traffic / alg, 4) if traffic else None,
            "tiles_key": tiles_key}


def nr_summary(hist, resid):
    import numpy as np
    it = np.arange(len(hist))
    tot = max(int(hist.sum()), 1)
    p99 = int(np.searchsorted(np.cumsum(hist), 0.99 * tot))
    return {"links": int(hist.sum()), "mean_iterations": round(float((hist * it).sum()) / tot, 3),
            "p99_iterations": p99, "max_final_residual": resid}


def run_suspension(steps):
    """The 256^3 periodic suspension of 200 bodies (seed 5, contact on),
    plain Newton."""
    import torch

    import paper_2209_10411_amd as mdl
    import workloads

    cfg = workloads.config5(seed=5)
    sim = mdl.Simulation(cfg, device="cuda:0")
    sim.step(5)
    sim.sync()
    sim.nr_histogram()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h, r = sim.nr_histogram()
    nc, nf = sim.contact_stats()
    sim.close()
    return dict(nr_summary(h, r), workload="256^3 periodic suspension, 200 bodies, contact, FP32, IBB", steps=steps,
                contacts=nc, contact_failures=nf,
                mlups=round(cfg.n_nodes * steps / dt / 1e6, 1), ms_per_step=round(dt * 1e3 / steps, 4))


def run_pair(steps, warmup, reps=3):
    """The two-body drafting workload (160x160x640 walls, 6- and 12-point
    bodies, contact) in its storage forms: FP32, FP16 and BF16 deviations."""
    import workloads

    out = {"workload": "two bodies 160x160x640 walls, tau 0.6, density ratio 1.2, g 2e-5, contact, IBB",
           "steps": steps}
    for name, st in (("f32", workloads.STORE_F32), ("f16", workloads.STORE_F16), ("bf16", workloads.STORE_BF16)):
        cfg = workloads.config3(storage=st)
        N = cfg.n_nodes
        dts, k_ms, k_n, k_nodes, _, _ = run_gpu(cfg, steps, warmup, reps)
        dt = median(dts)
        k_s = k_ms / 1e3 / max(k_n, 1)
        alg = k_nodes * bytes_per_node(st) + N
        ach = alg / k_s / 1e9
        traffic = traffic_from_profile(PMC_PAIR_SUMMARY, f"{name}_hbm_bytes_per_launch")
        out[name] = {"mlups": round(N * steps / dt / 1e6, 1), "ms_per_step": round(dt * 1e3 / steps, 5),
                     "kernel": (f"k_bulk_flat<{name}>" if cfg.nx % 64 else f"k_bulk<{name}>")
                     if st == workloads.STORE_F32 else f"k_bulk_pair<{name}>",
                     "kernel_avg_ms": round(k_ms / max(k_n, 1), 5), "kernel_achieved_GBs": round(ach, 1),
                     "kernel_frac": round(ach / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes_per_launch": int(alg),
                     "traffic": traffic, "traffic_over_algorithmic": round(traffic / alg, 4) if traffic else None}
    return out


def run_mlp_warmstart(steps, epochs):
    """Warm start on the 256^3 periodic suspension of 200 bodies (FP32,
    contact), evaluated on a system the network never saw: the MLP is
    trained on the link fractions the method solved at the initial
    geometries of seeds 6 and 7 and on the stationary points of their
    candidate body pairs over 10 steps (closest-point task), with Adam at a
    stepped learning rate (1e-3, then 3e-4, then 1e-4; `epochs` per stage);
    seed 5 then runs `steps` steps with plain and with warm-started Newton
    iterations from one checkpointed state (lbm_save / lbm_load), so both
    start from the same populations, poses and links.  Reported: training and
    held-out loss against the variance of q, Newton evaluations per link
    (mean, p99), pair solves and the step rate of both."""
    import tempfile

    import torch

    import paper_2209_10411_amd as mdl
    import workloads

    feats, targets = [], []
    t0 = time.perf_counter()
    n_contact = 0
    for seed in (6, 7):
        sim = mdl.Simulation(workloads.config5(seed=seed), device="cuda:0")
        f, t = mdl.mlp_collect(sim)
        feats.append(f.clone())
        targets.append(t.clone())
        for _ in range(10):
            sim.step(1)
            f, t = mdl.mlp_collect_contact(sim)
            # a few thousand pair samples against millions of link samples:
            # repeated to weigh the two tasks alike
            feats.append(f.repeat(100, 1))
            targets.append(t.repeat(100, 1))
            n_contact += int(f.shape[0])
        sim.close()
    sim5 = mdl.Simulation(workloads.config5(seed=5), device="cuda:0")
    hf, ht = mdl.mlp_collect(sim5)
    t_setup = time.perf_counter() - t0
    feat, target = torch.cat(feats), torch.cat(targets)
    perm = torch.randperm(feat.shape[0], generator=torch.Generator().manual_seed(0)).to(feat.device)
    feat, target = feat[perm].contiguous(), target[perm].contiguous()
    var_held = float(ht[:, 0].float().var())
    net = mdl.Mlp(workloads.mlp_init(5))
    _, loss0 = net.grad(feat[:4096], target[:4096])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lr in (1e-3, 3e-4, 1e-4):
        net.train(feat, target, lr=lr, epochs=epochs, batch=1024)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    _, loss1 = net.grad(feat[:4096], target[:4096])
    _, loss_held = net.grad(hf[:4096], ht[:4096])
    cfg = sim5.cfg
    sim5.step(5)
    ck = os.path.join(tempfile.mkdtemp(), "suspension.ckpt")
    sim5.save(ck)
    res = {}
    for mode in ("plain", "mlp"):
        sim5.load(ck)
        sim5.set_warmstart(net if mode == "mlp" else None)
        sim5.sync()
        sim5.nr_histogram()
        sim5.contact_nr_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim5.step(steps)
        sim5.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        h, r = sim5.nr_histogram()
        ns, ni = sim5.contact_nr_stats()
        res[mode] = dict(nr_summary(h, r), mlups=round(cfg.n_nodes * steps / dt / 1e6, 1),
                         ms_per_step=round(dt * 1e3 / steps, 4), pair_solves=ns,
                         pair_evaluations_per_solve=round(ni / max(ns, 1), 3),
                         contacts=sim5.contact_stats()[0])
    sim5.close()
    os.remove(ck)
    return {"workload": "256^3 periodic suspension, 200 bodies (6..20 cp, R 6..12), density ratio 1.5, "
                        "counter-force, contact, FP32, IBB; trained on seeds 6, 7, evaluated on seed 5",
            "training_samples": int(feat.shape[0]), "closest_point_samples": n_contact,
            "epochs_per_stage": epochs, "learning_rates": [1e-3, 3e-4, 1e-4], "batch": 1024,
            "train_s": round(t_train, 2), "setup_s": round(t_setup, 1),
            "loss_before": round(loss0, 5), "loss_after": round(loss1, 5), "held_out_loss": round(loss_held, 5),
            "held_out_var_q": round(var_held, 5), "steps": steps, "same_start": "lbm_save/lbm_load checkpoint",
            "plain": res["plain"], "mlp": res["mlp"]}


def run_fp16(steps, warmup, reps=3):
    """The same settling workload with FP16 deviation storage (the
    stream-collide in its node-pair form)."""
    import workloads
    cfg16 = workloads.config2()
    cfg16.storage = workloads.STORE_F16
    N = cfg16.n_nodes
    dts16, k16_ms, k16_n, k16_nodes, _, _ = run_gpu(cfg16, steps, warmup, reps)
    dt16 = median(dts16)
    k16_s = k16_ms / 1e3 / max(k16_n, 1)
    ach16 = (k16_nodes * bytes_per_node(1) + N) / k16_s / 1e9
    return {"value": round(N * steps / dt16 / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(dt16 * 1e3 / steps, 5), "kernel": "k_bulk_pair<f16>",
            "kernel_avg_ms": round(k16_ms / max(k16_n, 1), 5),
            "kernel_achieved_GBs": round(ach16, 1),
            "kernel_frac": round(ach16 / HBM_PEAK_GBS, 4)}


def kernel_source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def profile_values(path):
    """The key = value lines of a committed rocprofv3 --pmc summary, or None
    when it is missing or was taken on another kernel source."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_sha():
        return None
    return vals


def traffic_from_profile(path=None, key="hbm_bytes_per_launch"):
    """FETCH/WRITE bytes per launch of a stream-collide kernel from the
    committed rocprofv3 --pmc summary, if it was taken on this kernel source."""
    vals = profile_values(path or PMC_SUMMARY)
    try:
        return float(vals[key]) if vals else None
    except (KeyError, ValueError):
        return None


def run_mifit(ga_generations=100, gs_steps=200, gs_batch=256):
    """The Metaball-Imaging fit (sec. 2.2) with the paper's GA settings
    (E_ga = 100 generations, N_I = 1200 individuals, N_G = 100 genes = 25
    control points, C_m = 0.6, C_c = 0.5) on a synthetic hull of 4096 points
    sampled from a known 8-point metaball (R = 10), then the gradient search
    (eta = 1e-3) on a batch of such hulls, one workgroup per model; the GS
    steps are timed over a short run (the paper's E_gs = 1e5 per phase takes
    the same time per step).  Roofline of the fitness kernel: FP64 vector ALU,
    10 algorithmic flops per (hull point, control point) term (3
    differences, 3 products, 2 additions for |h - p|^2, one division, one
    addition) plus 3 per hull point ((f - 1)^2 and its sum)."""
    import numpy as np
    import torch

    import paper_2209_10411_amd as mdl
    import workloads

    dev = "cuda:0"
    cp, k = workloads.mi_body(seed=61, n_cp=8, R=10.0)
    H, pl, sh = workloads.mi_hull(cp, k, m=4096)
    N_I, n, E = 1200, 25, ga_generations
    pop0 = workloads.mi_population(H, pl, N_I, n, seed=62)
    U, Z, PERM = workloads.mi_draws(E, N_I, n, seed=63)
    sx, sk = 0.05 * float(np.abs(H).max()), 0.2 * float(pop0[..., 0].mean())
    truth = np.concatenate([k[:, None], cp - sh], 1)
    # the fitness kernel alone: 2 N_I individuals (one generation's offspring)
    L = mdl.lib()
    hd = torch.as_tensor(H, dtype=torch.float64, device=dev)
    popd = torch.as_tensor(np.concatenate([pop0, pop0]), dtype=torch.float64, device=dev)
    Fd = torch.empty(2 * N_I, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    wb = int(L.mi_fitness_work_bytes(len(H), 2 * N_I))
    wd = torch.empty(max(wb, 1), dtype=torch.uint8, device=dev)
    args = (C.c_void_p(hd.data_ptr()), len(H), C.c_void_p(popd.data_ptr()), 2 * N_I, n, C.c_void_p(Fd.data_ptr()),
            C.c_void_p(wd.data_ptr()), wb, C.c_void_p(stream.cuda_stream))
    for _ in range(3):
        if L.mi_fitness(*args) != 0:
            raise RuntimeError("mi_fitness failed")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        L.mi_fitness(*args)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = 2 * N_I * (10.0 * len(H) * n + 3.0 * len(H))
    # the whole GA
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pg, Fg = mdl.mi_ga(H, pop0, E, 0.6, 0.5, sx, sk, U, Z, PERM)
    t_ga = time.perf_counter() - t0
    # the gradient search on a batch of hulls from the GA's best model
    hulls, planes = [H] * gs_batch, [pl] * gs_batch
    M0 = np.repeat(pg[:1], gs_batch, axis=0)
    mdl.mi_gs(hulls[:1], planes[:1], M0[:1], 2, 1e-3)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Mg, Lg = mdl.mi_gs(hulls, planes, M0, gs_steps, 1e-3)
    t_gs = time.perf_counter() - t0
    return {"workload": "Metaball-Imaging fit, synthetic 4096-point hull of an 8-point metaball (R = 10); "
                        "GA E=100, N_I=1200, 25 control points, C_m=0.6, C_c=0.5; GS eta=1e-3",
            "fitness_kernel": {"individuals": 2 * N_I, "hull_points": len(H), "control_points": n,
                               "ms": round(ms, 4),
                               "roofline": {"bound": "alu", "achieved": round(flops / (ms * 1e-3) / 1e12, 2),
                                            "peak": 78.6, "unit": "TFLOP/s",
                                            "frac": round(flops / (ms * 1e-3) / 1e12 / 78.6, 4),
                                            "flops_per_launch": flops}},
            "ga": {"generations": E, "seconds": round(t_ga, 3), "ms_per_generation": round(t_ga * 1e3 / E, 3),
                   "best_fitness_initial": float(min(mdl.mi_fitness(H, pop0[:64]).min(), Fg.max())),
                   "best_fitness_final": float(Fg[0]), "truth_fitness": float(mdl.mi_fitness(H, truth[None])[0])},
            "gs": {"models": gs_batch, "steps_per_phase": gs_steps, "seconds": round(t_gs, 3),
                   "model_steps_per_s": round(gs_batch * 2 * gs_steps / t_gs, 1),
                   "s_per_model_at_1e5_steps_per_phase_batched": round(t_gs / (2 * gs_steps) * 2e5 / gs_batch, 3),
                   "loss": [float(v) for v in Lg[0]]}}


def dkt_matched_shapes(R=5.0, h=0.05):
    """Two-point bodies whose Corey shape factor, measured by the shape kernel,
    matches each of the paper's designed particles P1-P8 (bisection on the
    elongation a; the CSF falls monotonically with a)."""
    import paper_2209_10411_amd as mdl
    import workloads

    out = []
    for target in workloads.DKT_CSF_TARGETS:
        if target >= 1.0:
            out.append(workloads.dkt_body(0.0, R))
            continue
        lo, hi = 0.0, 0.98 * R
        for _ in range(14):
            mid = 0.5 * (lo + hi)
            if mdl.shape_descriptors(*workloads.dkt_body(mid, R), h)["CSF"] > target:
                lo = mid
            else:
                hi = mid
        out.append(workloads.dkt_body(0.5 * (lo + hi), R))
    return out


def run_dkt(steps=8000, every=25):
    """Drafting-kissing-tumbling of pairs of equal bodies with stepped
    elongation (sec. 4): two-point metaballs whose Corey shape factors match
    the paper's particles P1-P8 (dkt_matched_shapes), scaled to the volume of
    the sphere of radius 5 (D_e = 10 lu) with the volumes measured by the
    shape-descriptor kernel (grid step 0.05 before scaling), in a 160 x 160 x 240 walled box (the
    paper's container scaled to D_e), density ratio 2800/976, tau 0.55,
    gravity 1e-4 (settling Reynolds number near 20), contact on.  Per shape:
    sphericity, d_n/d_s, CSF from the GPU kernel, and from the coupled run
    (sampled every `every` steps) the closest approach of the centroids
    (kissing), the first step at which the trailing body is lower than the
    leading one (tumbling past), each body's peak settling speed and peak
    |omega| with their times, in the paper's units: time t_r = sqrt(H/g),
    velocity sqrt(H g), angular velocity 2 pi / t_r, distance D_e."""
    import numpy as np

    import paper_2209_10411_amd as mdl
    import workloads

    h = 0.05
    shapes = dkt_matched_shapes(h=h)
    d0 = mdl.shape_descriptors(*shapes[0], h)
    out = []
    t0 = time.perf_counter()
    for (cp, k), target in zip(shapes, workloads.DKT_CSF_TARGETS):
        d = mdl.shape_descriptors(cp, k, h)
        sc = (d0["V"] / d["V"]) ** (1.0 / 3.0)
        cp, k = cp * sc, k * sc * sc
        d = mdl.shape_descriptors(cp, k, h * sc)
        cfg = workloads.dkt_pair(cp, k)
        g = float(-cfg.g_particle[2])
        H = float(cfg.nz)
        tr, ur, wr = np.sqrt(H / g), np.sqrt(H * g), 2 * np.pi / np.sqrt(H / g)
        sim = mdl.Simulation(cfg, device="cuda:0")
        dmin, t_kiss, t_pass, done = 1e30, None, None, 0
        vmax, tv, wmax, tw = [0.0, 0.0], [0, 0], [0.0, 0.0], [0, 0]
        while done < steps:
            sim.step(every)
            done += every
            p = sim.particles()
            dist = float(np.linalg.norm(p[1]["x"] - p[0]["x"]))
            if dist < dmin:
                dmin, t_kiss = dist, done
            if t_pass is None and p[1]["x"][2] < p[0]["x"][2]:
                t_pass = done
            for b in range(2):
                v, w = -float(p[b]["v"][2]), float(np.linalg.norm(p[b]["omega"]))
                if v > vmax[b]:
                    vmax[b], tv[b] = v, done
                if w > wmax[b]:
                    wmax[b], tw[b] = w, done
            if min(p[0]["x"][2], p[1]["x"][2]) < 1.5 * d0["d_n"]:  # near the floor
                break
        nc, _ = sim.contact_stats()
        sim.close()
        out.append({"paper_CSF": target, "a": round(float(cp[1, 0]), 4), "Phi": round(d["Phi"], 4),
                    "dn_over_ds": round(d["d_n"] / d["d_s"], 4), "CSF": round(d["CSF"], 4),
                    "d_n": round(d["d_n"], 3), "steps_run": done,
                    "closest_centroid_distance_over_De": round(dmin / d0["d_n"], 3),
                    "t_closest_over_tr": round(t_kiss / tr, 4),
                    "t_trailing_passes_over_tr": round(t_pass / tr, 4) if t_pass else None,
                    "peak_settling_velocity_over_sqrtHg": [round(v / ur, 4) for v in vmax],
                    "t_peak_velocity_over_tr": [round(t / tr, 4) for t in tv],
                    "peak_angular_velocity_over_2pi_tr": [round(w / wr, 4) for w in wmax],
                    "t_peak_angular_velocity_over_tr": [round(t / tr, 4) for t in tw],
                    "contact_substeps": nc})
    return {"workload": "DKT pairs of equal-volume two-point metaballs with the CSF of the paper's P1-P8, "
                        "160x160x240 walls, D_e = 10 lu, density ratio 2.87, tau 0.55, g 1e-4, contact, IBB; "
                        "[leading, trailing] per pair",
            "steps": steps, "seconds": round(time.perf_counter() - t0, 1), "shapes": out}


GOLDEN = os.path.join(ROOT, "tests", "golden")


def trajectory_error(cfg, path):
    """The GPU run of cfg against the stored FP64 oracle trajectory at path
    (written by tests/golden/make_golden.py, which calls only the oracle):
    the largest particle |dx| over the stored samples and at the last one,
    and, where the file holds a field sample, max |du|/U and max |drho| over
    its fluid nodes (U = the oracle's max |u| over all fluid nodes)."""
    import numpy as np

    import paper_2209_10411_amd as mdl

    if not os.path.exists(path):
        return None
    g = np.load(path)
    steps, state = g["steps"], g["state"]
    fs = int(g["field_step"]) if "field_step" in g.files else None
    sim = mdl.Simulation(cfg, device="cuda:0")
    done, dxs, out = 0, [], {}
    for k, s in enumerate(steps):
        if fs is not None and done < fs <= s:
            sim.step(fs - done)
            done = fs
            rho, u = sim.macros()
            nodes = g["field_nodes"]
            fl = (g["field_owner"] < 0) & (sim.owner()[nodes] < 0)
            out["field_step"] = fs
            out["field_nodes"] = int(fl.sum())
            out["max_du_over_U"] = float(np.abs(u[nodes][fl] - g["field_u"][fl]).max() / float(g["field_umax"]))
            out["max_drho"] = float(np.abs(rho[nodes][fl] - g["field_rho"][fl]).max())
            del rho, u
        sim.step(int(s) - done)
        done = int(s)
        ps = sim.particles()
        dxs.append(max(float(np.abs(ps[j]["x"] - state[k, j, 0:3]).max()) for j in range(len(ps))))
    sim.close()
    out.update({"steps": int(steps[-1]), "samples": len(steps), "max_dx_lu": max(dxs), "final_dx_lu": dxs[-1],
                "dx_at": {str(int(steps[i])): dxs[i] for i in range(0, len(steps), max(1, len(steps) // 8))}})
    return out


def run_accuracy():
    """Error of each storage form against the stored FP64 oracle results:
    the settling workload (128x128x384, 2000 steps) in FP32 and FP16, and the
    two-body workload (160x160x640, 5000 steps; fields at step 200) in FP32,
    FP16 and BF16."""
    import workloads

    out = {"reference": "FP64 CPU oracle, stored by tests/golden/make_golden.py"}
    c2 = {}
    for name, st in (("f32", workloads.STORE_F32), ("f16", workloads.STORE_F16)):
        cfg = workloads.config2()
        cfg.storage = st
        c2[name] = trajectory_error(cfg, os.path.join(GOLDEN, "c2_trajectory.npz"))
    out["settling_128x128x384"] = c2
    c3 = {}
    for name, st in (("f32", workloads.STORE_F32), ("f16", workloads.STORE_F16), ("bf16", workloads.STORE_BF16)):
        c3[name] = trajectory_error(workloads.config3(storage=st), os.path.join(GOLDEN, "c3_trajectory.npz"))
    out["pair_160x160x640"] = c3
    return out


def cpu_model():
    """The host CPU's model name, or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(cfg, budget_s, min_steps=1):
    """Coupled oracle steps of cfg for about budget_s seconds: (MLUPS, steps,
    setup seconds)."""
    import oracle

    t0 = time.perf_counter()
    o = oracle.Oracle(cfg)
    t_init = time.perf_counter() - t0
    steps = 0
    t0 = time.perf_counter()
    while steps < min_steps or time.perf_counter() - t0 < budget_s:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    del o
    return cfg.n_nodes * steps / dt / 1e6, steps, t_init


def cpu_baseline(cfg, budget_s):
    """The FP64 oracle on the host: the settling case on every thread (the
    headline figure), the same case on one thread, and the 200-body
    suspension on every thread, each a bounded number of coupled steps."""
    import oracle

    nt = oracle.threads()
    v, steps, t_init = _oracle_rate(cfg, budget_s)
    out = {"value": round(v, 3), "unit": "MLUPS", "cores": nt, "kind": "oracle", "cpu": cpu_model(),
           "sample": f"{steps} coupled steps of the same 128x128x384 settling case "
                     f"(FP64, {nt} OpenMP threads, {t_init:.1f} s setup excluded)"}
    oracle.set_threads(1)
    try:
        v1, s1, _ = _oracle_rate(cfg, budget_s / 3)
    finally:
        oracle.set_threads(nt)
    out["single_thread"] = {"value": round(v1, 3), "unit": "MLUPS", "cores": 1,
                            "sample": f"{s1} coupled step(s) of the same settling case on one thread"}
    import workloads

    c5 = workloads.config5(seed=5)
    v5, s5, t5 = _oracle_rate(c5, budget_s / 2)
    out["suspension_256"] = {"value": round(v5, 3), "unit": "MLUPS", "cores": nt,
                             "sample": f"{s5} coupled step(s) of the 256^3 suspension of 200 bodies with contact "
                                       f"(FP64, {nt} threads, {t5:.1f} s setup excluded)"}
    return out


def copy_ceiling(n_nodes: int, reps: int = 20):
    """The library's streaming-copy probe (lbm_copy_probe): 19 FP32 arrays of
    n_nodes elements read and written with non-temporal stores, the
    stream-collide's access shape without its neighbour shifts and
    arithmetic; the practical ceiling of that kernel on this device.  None
    where it cannot be taken (no GPU)."""
    try:
        import paper_2209_10411_amd as mdl
        ms = mdl.copy_probe(n_nodes, 4, reps)
        gbs = 2 * 19 * 4 * n_nodes / (ms * 1e-3) / 1e9
        return {"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "ms": round(ms, 5),
                "kernel": "k_copy_soa<f32> (lbm_copy_probe)", "bytes_per_launch": 2 * 19 * 4 * n_nodes}
    except Exception:
        return None


def calib_copy(gib: float = 1.0):
    """A plain copy of known size, for scaling the PMC byte counters."""
    import torch
    n = int(gib * (1 << 30))
    a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": n, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--reps", type=int, default=5, help="timed regions of --steps steps (median reported)")
    ap.add_argument("--no-mifit", action="store_true", help="skip the Metaball-Imaging fit")
    ap.add_argument("--no-dkt", action="store_true", help="skip the drafting-kissing-tumbling shape sweep")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the comparison with the stored FP64 oracle trajectories")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-storage run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 64-case ensemble run")
    ap.add_argument("--ensemble-steps", type=int, default=60)
    ap.add_argument("--tune-cache", default=None, help="autotuner choices file for the ensemble (read or written)")
    ap.add_argument("--no-mlp", action="store_true", help="skip the warm-start (MLP) run")
    ap.add_argument("--mlp-steps", type=int, default=100)
    ap.add_argument("--mlp-epochs", type=int, default=4, help="epochs per learning-rate stage (three stages)")
    ap.add_argument("--calib-copy", action="store_true", help="only run a 1 GiB copy (PMC calibration)")
    ap.add_argument("--no-pair", action="store_true", help="skip the two-body 160x160x640 storage runs")
    ap.add_argument("--pair-steps", type=int, default=300)
    ap.add_argument("--only", choices=["ensemble", "warm-start", "suspension", "fp16", "pair", "accuracy", "mifit", "dkt"],
                    help="run only this part and print its JSON object (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by z-slabs across GPUs; that is not implemented)",
              file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy()
        return
    if args.only == "ensemble":
        print(json.dumps(run_ensemble(64, args.ensemble_steps, 12, args.tune_cache)), flush=True)
        return
    if args.only == "suspension":
        print(json.dumps(run_suspension(args.mlp_steps)), flush=True)
        return
    if args.only == "warm-start":
        print(json.dumps(run_mlp_warmstart(args.mlp_steps, args.mlp_epochs)), flush=True)
        return
    if args.only == "fp16":
        print(json.dumps(run_fp16(args.steps, args.warmup)), flush=True)
        return
    if args.only == "dkt":
        print(json.dumps(run_dkt()), flush=True)
        return
    if args.only == "mifit":
        print(json.dumps(run_mifit()), flush=True)
        return
    if args.only == "accuracy":
        print(json.dumps(run_accuracy()), flush=True)
        return
    if args.only == "pair":
        print(json.dumps(run_pair(args.pair_steps, args.warmup)), flush=True)
        return
    import workloads

    cfg = workloads.config2()
    N = cfg.n_nodes
    dts, k_ms, k_n, k_nodes, x, nr = run_gpu(cfg, args.steps, args.warmup, args.reps)
    dt = median(dts)
    mlups = N * args.steps / dt / 1e6
    k_avg_s = k_ms / 1e3 / max(k_n, 1)
    alg_bytes = k_nodes * bytes_per_node(0) + N  # populations of updated nodes + class byte of all
    achieved = alg_bytes / k_avg_s / 1e9
    traffic = traffic_from_profile()
    copy = copy_ceiling(N)
    out = {
        "metric": "MLUPS with moving metaball boundaries (FP32 vs FP16-store) + % HBM peak",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "settling-particle 128x128x384 walls, D3Q19 BGK tau=0.6, "
                               "1 metaball 8 cp R=10, density ratio 1.5, g=2e-5, IBB + refill, "
                               "FP32 deviation storage",
                   "nx": 128, "ny": 128, "nz": 384, "nodes": N, "storage": "f32",
                   "step": "coupled (links+MEM, rigid body, flags, stream-collide+refill, links)"},
        "timed_regions": {"count": len(dts), "steps_each": args.steps, "value": "median",
                          "ms_per_step": [round(t * 1e3 / args.steps, 5) for t in dts]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_bulk<f32>",
                     "target_frac": 0.70, "meets_target": achieved / HBM_PEAK_GBS >= 0.70,
                     "copy_ceiling": copy,
                     "frac_of_copy": round(achieved / copy["GBs"], 4) if copy else None,
                     "kernel_avg_ms": round(k_ms / max(k_n, 1), 5),
                     "kernel_launches_timed": k_n, "timed_every_nth_step": TIMING_EVERY,
                     "algorithmic_bytes_per_launch": alg_bytes},
        "kernel_mlups": round(k_nodes / k_avg_s / 1e6, 1),
        "particle_x_final": [round(v, 6) for v in x],
        "link_fraction_newton": {"links": nr[0], "mean_iterations": round(nr[1] / max(nr[0], 1), 3)},
    }
    if not args.no_fp16:
        out["fp16_store"] = run_fp16(args.steps, args.warmup)
    if not args.no_pair:
        out["pair_160x160x640"] = run_pair(args.pair_steps, args.warmup)
    if not args.no_ensemble:
        out["ensemble"] = run_ensemble(64, args.ensemble_steps, 12, args.tune_cache)
    if not args.no_mlp:
        out["warm_start"] = run_mlp_warmstart(args.mlp_steps, args.mlp_epochs)
    if not args.no_accuracy:
        out["accuracy"] = run_accuracy()
    if not args.no_mifit:
        out["metaball_imaging"] = run_mifit()
    if not args.no_dkt:
        out["dkt_shape_sweep"] = run_dkt()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
