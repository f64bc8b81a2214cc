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


def bytes_per_node(storage: int) -> int:
    return 19 * 2 * (4 if storage == 0 else 2)


def run_gpu(cfg, steps, warmup):
    import torch

    import paper_2209_10411_amd as mdl

    sim = mdl.Simulation(cfg, device="cuda:0")
    sim.step(warmup)
    sim.sync()
    sim.timing(True)
    sim.timing_read()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms, k_n, k_nodes = sim.timing_read()
    x = sim.particles()[0]["x"]
    nr = sim.nr_stats()
    sim.close()
    return dt, k_ms, k_n, k_nodes, x, nr


def run_ensemble(n_cases, steps, warmup):
    """The 64-case settling ensemble (random sizes 64..128 x 64..128 x 64..256,
    tau, density ratio, 4..16 control points; walls; FP32): autotuned tiles,
    batched launches with six-step graph replays, against the same systems
    stepped one after another with lbm_step."""
    import torch

    import paper_2209_10411_amd as mdl
    import workloads

    cfgs = workloads.config4(n_cases)
    nodes = sum(c.n_nodes for c in cfgs)
    ens = mdl.Ensemble(cfgs, device="cuda:0")
    t0 = time.perf_counter()
    tiles, bw = ens.autotune(budget_ms=5000.0)
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
    ens.close()
    return {"workload": f"{n_cases}-case settling ensemble, walls, FP32, 64..128 x 64..128 x 64..256, "
                        "tau U[0.55,1], density ratio U[1.1,2.5], 4..16 cp",
            "cases": n_cases, "nodes": nodes, "steps": steps,
            "value": round(nodes * steps / dt / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(dt * 1e3 / steps, 4),
            "unbatched_value": round(nodes * steps / dt_seq / 1e6, 1),
            "unbatched_ms_per_step": round(dt_seq * 1e3 / steps, 4),
            "tiles": hist, "waves_per_block": bw, "autotune_s": round(t_tune, 2)}


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


def run_pair(steps, warmup):
    """The two-body drafting workload (160x160x640 walls, 6- and 12-point
    bodies, contact) in its storage forms: FP32, FP16 and BF16 deviations."""
    import workloads

    out = {"workload": "two bodies 160x160x640 walls, tau 0.6, density ratio 1.2, g 2e-5, contact, IBB",
           "steps": steps}
    for name, st in (("f32", workloads.STORE_F32), ("f16", workloads.STORE_F16), ("bf16", workloads.STORE_BF16)):
        cfg = workloads.config3(storage=st)
        N = cfg.n_nodes
        dt, k_ms, k_n, k_nodes, _, _ = run_gpu(cfg, steps, warmup)
        k_s = k_ms / 1e3 / max(k_n, 1)
        ach = (k_nodes * bytes_per_node(st) + N) / k_s / 1e9
        out[name] = {"mlups": round(N * steps / dt / 1e6, 1), "ms_per_step": round(dt * 1e3 / steps, 5),
                     "kernel": "k_bulk<f32>" if st == workloads.STORE_F32 else
                     (f"k_bulk_pair<{name}>" if cfg.nx % 128 == 0 else f"k_bulk_pair_flat<{name}>"),
                     "kernel_avg_ms": round(k_ms / max(k_n, 1), 5), "kernel_achieved_GBs": round(ach, 1),
                     "kernel_frac": round(ach / HBM_PEAK_GBS, 4)}
    return out


def run_mlp_warmstart(steps, epochs):
    """Warm start on the 256^3 periodic suspension of 200 bodies (FP32,
    contact): the MLP is trained on the link fractions the method solved at
    the initial geometries of seeds 5, 6 and 7 and on the stationary points
    of the candidate body pairs over their first 10 steps (closest-point
    task), then seed 5 runs with plain and with warm-started Newton
    iterations (link fractions and pair solves)."""
    import torch

    import paper_2209_10411_amd as mdl
    import workloads

    feats, targets = [], []
    sim5 = None
    t0 = time.perf_counter()
    n_contact = 0
    for seed in (5, 6, 7):
        sim = mdl.Simulation(workloads.config5(seed=seed), device="cuda:0")
        f, t = mdl.mlp_collect(sim)
        feats.append(f.clone())
        targets.append(t.clone())
        if seed == 5:
            sim5 = sim
        else:
            for _ in range(10):
                sim.step(1)
                f, t = mdl.mlp_collect_contact(sim)
                # a few thousand pair samples against millions of link samples:
                # repeated to weigh the two tasks alike
                feats.append(f.repeat(100, 1))
                targets.append(t.repeat(100, 1))
                n_contact += int(f.shape[0])
            sim.close()
    t_setup = time.perf_counter() - t0
    feat, target = torch.cat(feats), torch.cat(targets)
    perm = torch.randperm(feat.shape[0], generator=torch.Generator().manual_seed(0)).to(feat.device)
    feat, target = feat[perm].contiguous(), target[perm].contiguous()
    net = mdl.Mlp(workloads.mlp_init(5))
    _, loss0 = net.grad(feat[:4096], target[:4096])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.train(feat, target, lr=1e-3, epochs=epochs, batch=1024)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    _, loss1 = net.grad(feat[:4096], target[:4096])
    cfg = sim5.cfg
    res = {}
    for mode in ("plain", "mlp"):
        sim5.set_warmstart(net if mode == "mlp" else None)
        sim5.step(5)
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
    return {"workload": "256^3 periodic suspension, 200 bodies (6..20 cp, R 6..12), density ratio 1.5, "
                        "counter-force, contact, FP32, IBB",
            "training_samples": int(feat.shape[0]), "closest_point_samples": n_contact, "epochs": epochs,
            "batch": 1024,
            "train_s": round(t_train, 2), "setup_s": round(t_setup, 1),
            "loss_before": round(loss0, 5), "loss_after": round(loss1, 5), "steps": steps,
            "plain": res["plain"], "mlp": res["mlp"]}


def run_fp16(steps, warmup):
    """The same settling workload with FP16 deviation storage (the
    stream-collide in its node-pair form)."""
    import workloads
    cfg16 = workloads.config2()
    cfg16.storage = workloads.STORE_F16
    N = cfg16.n_nodes
    dt16, k16_ms, k16_n, k16_nodes, _, _ = run_gpu(cfg16, steps, warmup)
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


def traffic_from_profile():
    """FETCH/WRITE bytes per launch of the stream-collide kernel from the
    committed rocprofv3 --pmc summary, if it was taken on this kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    sha = kernel_source_sha()
    vals = {}
    for line in open(PMC_SUMMARY):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != sha:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    """The host CPU's model name, or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, budget_s):
    import oracle

    t0 = time.perf_counter()
    o = oracle.Oracle(cfg)
    t_init = time.perf_counter() - t0
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    return {"value": round(cfg.n_nodes * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": oracle.threads(),
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{steps} coupled steps of the same 128x128x384 settling case "
                      f"(FP64, {oracle.threads()} OpenMP threads, {t_init:.1f} s setup excluded)"}


def copy_achievable(gib: float = 1.0, reps: int = 10):
    """Bandwidth of a plain device-to-device copy (GB/s, bytes read plus
    written), timed with events on torch's stream: the practical ceiling of a
    streaming kernel on this machine, reported beside the published peak.  None
    where it cannot be taken (no GPU)."""
    try:
        import torch
        n = int(gib * (1 << 30))
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        del a, b
        torch.cuda.empty_cache()
        return round(2 * n / (ms * 1e-3) / 1e9, 1)
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
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-storage run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 64-case ensemble run")
    ap.add_argument("--ensemble-steps", type=int, default=60)
    ap.add_argument("--no-mlp", action="store_true", help="skip the warm-start (MLP) run")
    ap.add_argument("--mlp-steps", type=int, default=100)
    ap.add_argument("--mlp-epochs", type=int, default=3)
    ap.add_argument("--calib-copy", action="store_true", help="only run a 1 GiB copy (PMC calibration)")
    ap.add_argument("--no-pair", action="store_true", help="skip the two-body 160x160x640 storage runs")
    ap.add_argument("--pair-steps", type=int, default=300)
    ap.add_argument("--only", choices=["ensemble", "warm-start", "suspension", "fp16", "pair"],
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
        print(json.dumps(run_ensemble(64, args.ensemble_steps, 12)), flush=True)
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
    if args.only == "pair":
        print(json.dumps(run_pair(args.pair_steps, args.warmup)), flush=True)
        return
    import workloads

    cfg = workloads.config2()
    N = cfg.n_nodes
    dt, k_ms, k_n, k_nodes, x, nr = run_gpu(cfg, args.steps, args.warmup)
    mlups = N * args.steps / dt / 1e6
    k_avg_s = k_ms / 1e3 / max(k_n, 1)
    alg_bytes = k_nodes * bytes_per_node(0) + N  # populations of updated nodes + class byte of all
    achieved = alg_bytes / k_avg_s / 1e9
    traffic = traffic_from_profile()
    copy_gbs = copy_achievable()
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
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_bulk<f32>",
                     "copy_achievable_GBs": copy_gbs,
                     "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None,
                     "kernel_avg_ms": round(k_ms / max(k_n, 1), 5),
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
        out["ensemble"] = run_ensemble(64, args.ensemble_steps, 12)
    if not args.no_mlp:
        out["warm_start"] = run_mlp_warmstart(args.mlp_steps, args.mlp_epochs)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
