"""Benchmark of the coupled LBM-DEM hot path on one MI355X.

Workload: the drop-sweeping-particles configuration (256x128x96 lattice, drop of
radius 30 pushed along x by a body force 5e-6 over a 110-degree wall, 20 spheres
of radius 5), FP32 population storage.  A step is one whole coupled time step:
collide-recolour-stream + bounce-back + momentum exchange, capillary force,
DEM, mask update, refill and order parameter.

Prints one JSON line: throughput in MLUPS (all lattice nodes per step), the
roofline of the dominant kernel (k_fused, HBM-bound) from HIP events recorded
inside the timed steps, and the FP64 CPU oracle timed on a bounded sample of the
same workload on this host.
"""
import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (f+g+particles) & % HBM peak; ensemble runs/hour at ≤1e-3 error"
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "k_fused_drop_sweep_256x128x96_fp32_counters.txt")


def traffic_from_profile():
    """HBM bytes per k_fused launch from the committed rocprofv3 counter
    summary, or None if it is missing or was taken on different kernel sources."""
    from paper_2505_10171_amd.prof_summary import kernel_sources_hash
    if not os.path.exists(COUNTERS):
        return None
    txt = open(COUNTERS).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_sources_hash():
        return None
    return float(b.group(1))


def cpu_baseline(work, steps):
    from oracle import oracle as O
    from oracle.oracle import OracleSim
    t0 = time.perf_counter()
    sim = OracleSim(work["cfg"], work["phi0"], work["particles"])
    t1 = time.perf_counter()
    sim.step(steps)
    t2 = time.perf_counter()
    N = work["cfg"]["nx"] * work["cfg"]["ny"] * work["cfg"]["nz"]
    sim.close()
    return dict(value=N * steps / (t2 - t1) / 1e6, unit="MLUPS", cores=O.num_threads(),
                kind="oracle",
                sample=f"first {steps} steps of the same workload (FP64 oracle, OpenMP, "
                       f"{t2 - t1:.1f} s; setup {t1 - t0:.1f} s excluded)")


def ensemble(args):
    """Batched ensemble of C4 members (uneven cubic boxes, one sphere each) in
    one context: every phase one launch over all members, pairs of steps
    replayed from a HIP graph.  runs/hour = members x 3600 / wall time of one
    full run (5,000 steps; timed whole by default, with --steps K the K-step
    time is scaled by 5000/K).  The error gate re-runs the two smallest members
    of the same storage type against the FP64 oracle for --gate-steps steps:
    max relative L2 of u and phi <= 1e-3."""
    import numpy as np
    import torch
    from paper_2505_10171_amd import workloads as W
    from paper_2505_10171_amd.lbm import Context
    members = [W.ensemble_member_c4(4, i, storage=args.storage) for i in range(args.members)]
    run_steps = members[0]["steps"]  # one run of every member
    steps = args.steps if args.steps_given else run_steps
    nodes = sum(m["cfg"]["nx"] * m["cfg"]["ny"] * m["cfg"]["nz"] for m in members)
    stream = torch.cuda.Stream()
    ctx = Context(members, stream=stream)
    ctx.use_graph(True)
    ctx.step(args.warmup + (args.warmup % 2))
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    wall = t1 - t0
    # error gate on the two smallest members
    from oracle.oracle import OracleSim
    order = sorted(range(len(members)), key=lambda i: members[i]["cfg"]["nx"])[:2]
    gate = []
    for i in order:
        m = members[i]
        g = Context([m])
        g.step(args.gate_steps)
        o = OracleSim(dict(m["cfg"], storage="fp32"), m["phi0"], m["particles"])
        o.step(args.gate_steps)
        rg, ug, pg, mg = g.fields()
        ro, uo, po, mo = o.fields()
        fl = mo == 0
        eu = float(np.linalg.norm(ug[:, fl] - uo[:, fl]) / np.linalg.norm(uo[:, fl]))
        ep = float(np.linalg.norm(pg[fl] - po[fl]) / np.linalg.norm(po[fl]))
        gate.append(dict(member=i, L=m["cfg"]["nx"], u=eu, phi=ep))
        g.close()
        o.close()
    ok = all(max(e["u"], e["phi"]) <= 1e-3 for e in gate)
    out = {
        "metric": "ensemble runs/hour at <=1e-3 error",
        "value": round(args.members * 3600.0 / (wall / steps * run_steps), 1) if ok else 0.0,
        "unit": "runs/hour", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ensemble of {args.members} cubic boxes L in {{48,64,80,96}}, "
                               f"one sphere each, {args.storage.upper()} storage",
                   "members": args.members, "nodes": nodes, "storage": args.storage},
        "mlups": round(nodes * steps / wall / 1e6, 1), "steps_per_run": run_steps,
        "gate": {"steps": args.gate_steps, "members": gate, "passed": ok},
    }
    print(json.dumps(out), flush=True)


def scale_c3(args):
    """The 512x256x192 slab workload with 500 spheres, FP32 and FP16 storage on
    the same run: MLUPS of each, the roofline of k_fused for each, and the
    per-field error of FP16 against FP32 after the timed steps; both against
    the FP64 oracle after --c3-oracle-steps steps."""
    import numpy as np
    import torch
    from paper_2505_10171_amd import workloads as W
    from paper_2505_10171_amd.lbm import Simulation

    def rel(a, b):
        return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))

    res = {}
    fields = {}
    for storage in ("fp32", "fp16"):
        w = W.slab_c3(storage=storage)
        cfg = w["cfg"]
        N = cfg["nx"] * cfg["ny"] * cfg["nz"]
        sim = Simulation(cfg, w["phi0"], w["particles"])
        n_fluid = int((sim.phi_mask()[1] == 0).sum())
        sim.step(args.warmup)
        sim.sync()
        sim.profile(True, every=10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(args.steps)
        sim.sync()
        t1 = time.perf_counter()
        prof = sim.profile_read()
        sim.profile(False)
        pop_b, ref_b = (2, 8) if storage == "fp16" else (4, 0)
        alg = n_fluid * (38 * pop_b + 24 + ref_b) + (N - n_fluid) * 8
        t_f = prof["fused"][0] / max(prof["fused"][1], 1) * 1e-3
        res[storage] = {"mlups": round(N * args.steps / (t1 - t0) / 1e6, 1),
                        "ms_per_step": round((t1 - t0) * 1e3 / args.steps, 4),
                        "k_fused_gbs": round(alg / t_f / 1e9, 1),
                        "k_fused_frac": round(alg / t_f / (HBM_PEAK_GBS * 1e9), 4),
                        "phase_ms_per_step": {k: round(v[0] / max(v[1], 1), 5)
                                              for k, v in prof.items()}}
        r, u, phi, mask = sim.fields()
        fields[storage] = (r, u, phi, mask)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    a, b = fields["fp16"], fields["fp32"]
    fl = b[3] == 0
    res["fp16_vs_fp32_after_timed_steps"] = {
        "rho": rel(a[0][fl], b[0][fl]), "u": rel(a[1][:, fl], b[1][:, fl]),
        "phi": rel(a[2][fl], b[2][fl]), "masks_equal": bool(np.array_equal(a[3], b[3]))}
    if args.c3_oracle_steps > 0:
        from oracle.oracle import OracleSim
        w = W.slab_c3()
        o = OracleSim(w["cfg"], w["phi0"], w["particles"])
        o.step(args.c3_oracle_steps)
        ro, uo, po, mo = o.fields()
        o.close()
        fl = mo == 0
        for storage in ("fp32", "fp16"):
            w = W.slab_c3(storage=storage)
            sim = Simulation(w["cfg"], w["phi0"], w["particles"])
            sim.step(args.c3_oracle_steps)
            r, u, phi, mask = sim.fields()
            sim.close()
            del sim
            torch.cuda.empty_cache()
            res[f"{storage}_vs_oracle_{args.c3_oracle_steps}_steps"] = {
                "rho": rel(r[fl], ro[fl]), "u": rel(u[:, fl], uo[:, fl]),
                "phi": rel(phi[fl], po[fl]), "masks_equal": bool(np.array_equal(mask, mo))}
    out = {"metric": "MLUPS (f+g+particles), FP32 vs FP16 storage", "value": res["fp32"]["mlups"],
           "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "liquid slab 512x256x192, 500 spheres R=4"}, "c3": res}
    print(json.dumps(out), flush=True)


def surrogate(args):
    """The surrogate trained on runs of the coupled method (committed data set of
    4,096 training and 256 held-out runs of the uneven-box distribution) and
    checked against the held-out plain runs.  Effective runs/hour: the plain
    ensemble rate (timed here on 256 members) divided by the fraction of runs
    the surrogate hands back to the plain method (confidence below 0.9), plus
    its own inference time."""
    import torch
    from paper_2505_10171_amd import surrogate_eval as E
    train = E.load(E.TRAIN_FILES)
    held = E.load(E.HELDOUT_FILES)
    res = E.train_and_evaluate(train, held, epochs=args.srg_epochs)
    # plain method rate on the same GPU: the batched ensemble
    from paper_2505_10171_amd import workloads as W
    from paper_2505_10171_amd.lbm import Context
    members = [W.ensemble_member_c4(4, i) for i in range(256)]
    ctx = Context(members, stream=torch.cuda.Stream())
    ctx.use_graph(True)
    ctx.step(4)
    ctx.sync()
    t0 = time.perf_counter()
    ctx.step(200)
    ctx.sync()
    ms_step = (time.perf_counter() - t0) * 1e3 / 200
    ctx.close()
    plain_rph = 256 * 3600.0 / (ms_step * 1e-3 * 5000)
    n = len(held["label"])
    f = res["fallback_fraction"]
    t_surr = res["infer_us"] * 1e-6 * max(1.0, n / res["infer_batch"])
    eff_rph = n * 3600.0 / (t_surr + f * n * 3600.0 / plain_rph)
    out = {
        "metric": "surrogate effective runs/hour with fallback (held-out plain runs as truth)",
        "value": round(eff_rph, 1), "unit": "runs/hour", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "MLP 6-256x4-51 on 4,096 runs of the uneven-box ensemble, "
                               "256 held-out runs", "epochs": args.srg_epochs},
        "plain_runs_per_hour": round(plain_rph, 1),
        "roofline": {"bound": "mfma", "achieved": res["infer_tflops"], "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(res["infer_tflops"] / 2500.0, 5),
                     "kernel": "k_mlp (inference, batch %d)" % res["infer_batch"],
                     "traffic": None},
        "surrogate": res,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16"])
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter scaling)")
    ap.add_argument("--ensemble", action="store_true",
                    help="batched ensemble of uneven boxes (runs/hour) instead of the drop sweep")
    ap.add_argument("--members", type=int, default=256)
    ap.add_argument("--gate-steps", type=int, default=20)
    ap.add_argument("--surrogate", action="store_true",
                    help="train and evaluate the surrogate on the committed runs of the method")
    ap.add_argument("--srg-epochs", type=int, default=200)
    ap.add_argument("--c3", action="store_true",
                    help="512x256x192 slab with 500 spheres, FP32 vs FP16 storage")
    ap.add_argument("--c3-oracle-steps", type=int, default=20)
    args = ap.parse_args()
    args.steps_given = any(a.startswith("--steps") for a in sys.argv[1:])
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    if args.ensemble:
        return ensemble(args)
    if args.surrogate:
        return surrogate(args)
    if args.c3:
        return scale_c3(args)
    import torch
    from paper_2505_10171_amd import workloads as W
    from paper_2505_10171_amd.lbm import Simulation

    work = W.drop_sweep_c2()
    work["cfg"]["storage"] = args.storage
    cfg = work["cfg"]
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    sim = Simulation(cfg, work["phi0"], work["particles"])
    rho, u, phi, mask = sim.fields()
    n_fluid = int((mask == 0).sum())
    sim.step(args.warmup)
    sim.sync()

    # HIP events around the phases of every 10th step of the timed region
    # (events on every step would add about 4 % to the step time)
    sim.profile(True, every=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_read()
    sim.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    mlups = N * args.steps / (t1 - t0) / 1e6

    # algorithmic bytes of one k_fused launch.  Per fluid node: the 19 stored
    # populations read and written once (4 B each, 2 B in FP16 storage; the
    # colour is not stored), the interface normal (12 B), the curvature term +
    # solid-link word (8 B) and phi (4 B) read; FP16 adds the reference
    # densities: the node's previous one for decoding (4 B) and the current one
    # of the nodes written to (4 B per node).  Per solid node the link word.
    pop_b = 2 if args.storage == "fp16" else 4
    ref_b = 8 if args.storage == "fp16" else 0
    alg_bytes = n_fluid * (38 * pop_b + 12 + 8 + 4 + ref_b) + (N - n_fluid) * 8
    fused_ms, fused_n = prof["fused"]
    t_fused = fused_ms / max(fused_n, 1) * 1e-3
    achieved = alg_bytes / t_fused / 1e9
    traffic = traffic_from_profile() if args.storage == "fp32" else None
    # whole-step effective fraction: B_alg per node-step (populations read and
    # written by the collision and read by the moments pass, moments written,
    # mask read) at the measured MLUPS
    b_alg_node = 19 * pop_b * 3 + 8 + 2
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"drop sweeping particles 256x128x96, 20 spheres R=5, "
                               f"{args.storage.upper()} population storage",
                   "lattice": [cfg["nx"], cfg["ny"], cfg["nz"]], "particles": 20,
                   "storage": args.storage, "global_batch": 1},
        "roofline": {"bound": "hbm", "kernel": "k_fused",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": round(t_fused * 1e3, 5)},
        "phase_ms_per_step": {k: round(v[0] / max(v[1], 1), 5) for k, v in prof.items()},
        "hbm_effective_frac": round(mlups * 1e6 * b_alg_node / (HBM_PEAK_GBS * 1e9), 4),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(work, args.cpu_steps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
