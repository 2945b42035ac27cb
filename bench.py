"""Benchmark of the coupled LBM-DEM hot path on one MI355X.

The line's workload is the throughput-at-scale configuration: a 512x256x192
lattice (25.2 M nodes) with a liquid slab filling 40 % of the height over a
90-degree wall and 500 spheres of radius 4, FP32 population storage.  A step is
one whole coupled time step: interface normal and curvature, collide-stream
with bounce-back, momentum exchange on particle links, capillary force, DEM,
mask update, refill and the order parameter of the new state.

One JSON line:
- value: MLUPS (all lattice nodes per step) of the FP32 run;
- roofline: the fused-step group (k_interface, k_fused, k_links, k_moments:
  the population and interface traffic of the step) against the method's
  algorithmic bytes per node-step, 314 B in FP32 (every population of f and g
  read and written once, phi written and read once, the mask read once), from
  HIP events recorded on the library's stream inside the timed steps, with a
  sub-entry per kernel against its own bytes;
- fp16: the same run with FP16 population storage (162 B per node-step), and
  its fields' distance to the FP32 run after the timed steps;
- c2: the 256x128x96 drop-sweep workload (20 spheres), FP32;
- c4: the batched ensemble of 256 uneven cubic boxes, runs per hour of
  5,000-step runs, with graph replay;
- table1: the paper's own drop-particle run (Table 1: 400x181x71, R_p = 10,
  drop radius 5 R_p, viscosity ratio 10), FP32;
- tube: the hydrodynamic-force benchmark's set-up (a sphere of radius 12.2 in
  pressure-driven flow through a tube of radius 40 between anti-bounce-back
  pressure ends, 320x83x83), FP32;
- textured: a drop on a textured wall (eight pillars) with six spheres,
  256x128x64, FP32;
- cpu_baseline: the FP64 oracle timed on a bounded sample of the same workload
  on this host's cores (all usable threads, and one thread), and, from the same
  oracle runs, the GPU fields' error at the sampled step counts (the C3 sample
  and one ensemble member of each box side).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (f+g+particles) & % HBM peak; ensemble runs/hour at ≤1e-3 error"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per node-step of the method (both population sets read and
# written once, phi written and read once, the uint16 mask read once)
B_ALG = {"fp32": 314, "fp16": 162}
GROUP = ("interface", "fused", "links", "moments")
COUNTERS = {"fp32": os.path.join(ROOT, "profiles",
                                 "fused_group_slab_512x256x192_fp32_counters.txt")}
GROUP_KERNELS = ("k_interface", "k_fused<", "k_links<", "k_moments<")


def kernel_bytes(storage, N, n_fluid):
    """Algorithmic bytes per launch of each timed phase of the group, each
    counting what that kernel must read and write once:
    interface (k_interface): phi read, the normal (3 components + |G|) and
        the CSF coefficient with the solid-link word written: 4 + 16 + 8 = 28 B
        per node;
    fused: per fluid node the 19 stored populations read and written (4 B
        each, 2 B in FP16), the normal (12 B), the curvature word (8 B) and phi
        (4 B); FP16 adds the two reference densities (8 B); per solid node the
        curvature word (8 B);
    moments: the 19 populations read, the colliding state's (rho, phi, normal)
        read (20 B), the mask (2 B), the new (rho, phi) written (8 B).
    k_links has O(particle links) work and no per-node bytes."""
    p = 2 if storage == "fp16" else 4
    ref = 8 if storage == "fp16" else 0
    return {"interface": 28 * N,
            "fused": n_fluid * (38 * p + 24 + ref) + (N - n_fluid) * 8,
            "moments": N * (19 * p + 20 + 2 + 8),
            "links": None}


def traffic_from_profile(storage):
    """Measured HBM bytes per step of the group kernels from the committed
    rocprofv3 counter summary, or None if absent or taken on other sources."""
    from paper_2505_10171_amd.prof_summary import kernel_sources_hash, read_counters
    path = COUNTERS.get(storage)
    if not path or not os.path.exists(path):
        return None
    per, h = read_counters(path)
    if h != kernel_sources_hash():
        return None
    tot = 0.0
    for k in GROUP_KERNELS:
        hits = [v for name, v in per.items() if k in name]
        if not hits:
            return None
        tot += hits[0]
    return tot


def run_lattice(work, steps, warmup):
    """Time `steps` steps after `warmup`; phases from HIP events every 10th step."""
    import torch
    from paper_2505_10171_amd.lbm import Simulation
    cfg = work["cfg"]
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]
    sim = Simulation(cfg, work["phi0"], work["particles"])
    n_fluid = int((sim.phi_mask()[1] == 0).sum())
    sim.step(warmup)
    sim.sync()
    sim.profile(True, every=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_read()
    sim.profile(False)
    fields = sim.fields()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    ph = {k: v[0] / max(v[1], 1) for k, v in prof.items()}  # ms per step
    storage = cfg["storage"]
    kb = kernel_bytes(storage, N, n_fluid)
    group_ms = sum(ph[k] for k in GROUP)
    alg = B_ALG[storage] * N
    kernels = {}
    for k in GROUP:
        e = {"avg_ms": round(ph[k], 5)}
        if kb[k] is not None:
            gbs = kb[k] / (ph[k] * 1e-3) / 1e9
            e.update(alg_bytes=kb[k], achieved_gbs=round(gbs, 1),
                     frac=round(gbs / HBM_PEAK_GBS, 4))
        kernels[k] = e
    achieved = alg / (group_ms * 1e-3) / 1e9
    mlups = N * steps / (t1 - t0) / 1e6
    traffic = traffic_from_profile(storage)
    roof = {"bound": "hbm",
            "kernel": "fused-step group: k_interface + k_fused + k_links + k_moments",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "alg_bytes_per_launch": alg, "alg_bytes_per_node": B_ALG[storage],
            "avg_launch_ms": round(group_ms, 5), "kernels": kernels}
    return dict(N=N, n_fluid=n_fluid, mlups=mlups, ms_per_step=(t1 - t0) * 1e3 / steps,
                phases=ph, roofline=roof, fields=fields,
                hbm_effective_frac=mlups * 1e6 * B_ALG[storage] / (HBM_PEAK_GBS * 1e9))


def rel(a, b):
    import numpy as np
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def field_errors(f, ref):
    import numpy as np
    fl = (ref[3] == 0) & (f[3] == 0)
    return {"rho": rel(f[0][fl], ref[0][fl]), "u": rel(f[1][:, fl], ref[1][:, fl]),
            "phi": rel(f[2][fl], ref[2][fl]), "masks_equal": bool(np.array_equal(f[3], ref[3]))}


def gpu_fields_after(work, steps, sim=None):
    """GPU fields of a fresh run of `steps` steps (one simulation or, with
    sim, member `sim` of an ensemble context already stepped)."""
    import torch
    from paper_2505_10171_amd.lbm import Simulation
    s = Simulation(work["cfg"], work["phi0"], work["particles"])
    s.step(steps)
    f = s.fields()
    s.close()
    del s
    torch.cuda.empty_cache()
    return f


def ensemble(n_members, steps, warmup, storage="fp32"):
    """The batched ensemble (uneven cubic boxes, one sphere each) in one
    context, every phase one launch over all members, pairs of steps replayed
    from a HIP graph.  runs/hour = members x 3600 / (time per step x 5,000).
    Returns the rate and, per box side, the fields of the first member of that
    side after warmup + steps steps (for the error gate)."""
    import torch
    from paper_2505_10171_amd import workloads as W
    from paper_2505_10171_amd.lbm import Context
    members = [W.ensemble_member_c4(4, i, storage=storage) for i in range(n_members)]
    run_steps = members[0]["steps"]
    nodes = sum(m["cfg"]["nx"] * m["cfg"]["ny"] * m["cfg"]["nz"] for m in members)
    ctx = Context(members, stream=torch.cuda.Stream())
    ctx.use_graph(True)
    warmup += warmup % 2
    ctx.step(warmup)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gate = {}
    for i, m in enumerate(members):
        L = m["cfg"]["nx"]
        if L not in gate:
            gate[L] = (i, ctx.fields(i))
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return dict(members=n_members, nodes=nodes, steps=steps, run_steps=run_steps,
                ms_per_step=wall * 1e3 / steps, mlups=nodes * steps / wall / 1e6,
                runs_per_hour=n_members * 3600.0 / (wall / steps * run_steps),
                gate_fields=gate, gate_steps=warmup + steps, storage=storage)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(c3_work, c3_steps, c3_gpu_fields, c4):
    """The FP64 oracle, unchanged, on this host: the first c3_steps steps of the
    C3 workload with all usable threads, then one more step on one thread;
    from the same oracle runs, the GPU's error at those step counts: the C3
    FP32 fields, and the ensemble's gate members (one per box side) after the
    ensemble's warm-up and timed steps, within 1e-3 in u and phi."""
    from oracle import oracle as O
    from oracle.oracle import OracleSim
    from paper_2505_10171_amd import workloads as W
    threads = len(os.sched_getaffinity(0))
    O.set_num_threads(threads)
    N = c3_work["cfg"]["nx"] * c3_work["cfg"]["ny"] * c3_work["cfg"]["nz"]
    t0 = time.perf_counter()
    sim = OracleSim(c3_work["cfg"], c3_work["phi0"], c3_work["particles"])
    t1 = time.perf_counter()
    sim.step(c3_steps)
    t2 = time.perf_counter()
    err_c3 = field_errors(c3_gpu_fields, sim.fields())
    O.set_num_threads(1)
    t3 = time.perf_counter()
    sim.step(1)
    t4 = time.perf_counter()
    O.set_num_threads(threads)
    sim.close()
    multi = N * c3_steps / (t2 - t1) / 1e6
    single = N / (t4 - t3) / 1e6
    gate = []
    for L, (i, f) in sorted(c4["gate_fields"].items()):
        m = W.ensemble_member_c4(4, i)
        o = OracleSim(m["cfg"], m["phi0"], m["particles"])
        o.step(c4["gate_steps"])
        e = field_errors(f, o.fields())
        o.close()
        gate.append(dict(member=i, L=L, u=e["u"], phi=e["phi"]))
    return dict(
        value=round(multi, 3), unit="MLUPS", cores=threads, kind="oracle",
        sample=f"first {c3_steps} steps of the 512x256x192 slab with 500 spheres (FP64 oracle, "
               f"OpenMP, {t2 - t1:.1f} s; setup {t1 - t0:.1f} s excluded); one more step on one "
               f"thread {t4 - t3:.1f} s",
        single_thread_mlups=round(single, 4), cpu_model=cpu_model(),
        gpu_error_c3_fp32=err_c3,
        ensemble_gate={"steps": c4["gate_steps"], "members": gate,
                       "passed": all(max(g["u"], g["phi"]) <= 1e-3 for g in gate)})


def surrogate(args):
    """The surrogate trained on runs of the coupled method (committed data set of
    4,096 training and 256 held-out runs of the uneven-box distribution) and
    checked against the held-out plain runs.  Effective runs/hour: the plain
    ensemble rate (timed here on 256 members) divided by the fraction of runs
    the surrogate hands back to the plain method (confidence below 0.9), plus
    its own inference time."""
    from paper_2505_10171_amd import surrogate_eval as E
    train = E.load(E.TRAIN_FILES)
    held = E.load(E.HELDOUT_FILES)
    res = E.train_and_evaluate(train, held, epochs=args.srg_epochs)
    c4 = ensemble(256, 200, 4)
    plain_rph = c4["runs_per_hour"]
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
    ap.add_argument("--steps", type=int, default=500, help="timed steps of the C3 runs")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--only", choices=["c3", "c3-fp16", "c2", "c4", "table1", "tube", "textured"],
                    default=None,
                    help="run one part alone (for profiling): no line, a short summary")
    ap.add_argument("--c2-steps", type=int, default=2000)
    ap.add_argument("--c4-steps", type=int, default=200)
    ap.add_argument("--table1-steps", type=int, default=2000)
    ap.add_argument("--tube-steps", type=int, default=2000)
    ap.add_argument("--textured-steps", type=int, default=2000)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter scaling)")
    ap.add_argument("--surrogate", action="store_true",
                    help="train and evaluate the surrogate on the committed runs of the method")
    ap.add_argument("--srg-epochs", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU slab "
              "decomposition is described, not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2505_10171_amd import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.surrogate:
        return surrogate(args)
    if args.only:
        if args.only in ("c3", "c3-fp16"):
            r = run_lattice(W.slab_c3(storage="fp16" if args.only == "c3-fp16" else "fp32"),
                            args.steps, args.warmup)
        elif args.only == "c2":
            r = run_lattice(W.drop_sweep_c2(), args.steps, args.warmup)
        elif args.only == "table1":
            r = run_lattice(W.table1_n1(), args.steps, args.warmup)
        elif args.only == "tube":
            r = run_lattice(W.tube_segre(), args.steps, args.warmup)
        elif args.only == "textured":
            r = run_lattice(W.textured_wall(), args.steps, args.warmup)
        else:
            r = ensemble(256, args.c4_steps, 4)
            r.pop("gate_fields")
            print(json.dumps(r), flush=True)
            return
        r.pop("fields")
        print(json.dumps({k: r[k] for k in ("mlups", "ms_per_step", "roofline", "phases")}),
              flush=True)
        return

    c3w = W.slab_c3()
    r32 = run_lattice(c3w, args.steps, args.warmup)
    r16 = run_lattice(W.slab_c3(storage="fp16"), args.steps, args.warmup)
    e16 = field_errors(r16["fields"], r32["fields"])
    r2 = run_lattice(W.drop_sweep_c2(), args.c2_steps, 20)
    c4 = ensemble(256, args.c4_steps, 4)
    rt1 = run_lattice(W.table1_n1(), args.table1_steps, 20)
    rtb = run_lattice(W.tube_segre(), args.tube_steps, 20)
    rtx = run_lattice(W.textured_wall(), args.textured_steps, 20)
    cfg = c3w["cfg"]
    out = {
        "metric": METRIC,
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "liquid slab 512x256x192 (40% of the height), 500 spheres R=4, "
                               "90-degree wall, FP32 population storage",
                   "lattice": [cfg["nx"], cfg["ny"], cfg["nz"]], "particles": 500,
                   "storage": "fp32", "global_batch": 1},
        "roofline": r32["roofline"],
        "hbm_effective_frac": round(r32["hbm_effective_frac"], 4),
        "phase_ms_per_step": {k: round(v, 5) for k, v in r32["phases"].items()},
        "fp16": {"mlups": round(r16["mlups"], 1), "ms_per_step": round(r16["ms_per_step"], 5),
                 "speedup_vs_fp32": round(r16["mlups"] / r32["mlups"], 3),
                 "roofline": r16["roofline"],
                 "hbm_effective_frac": round(r16["hbm_effective_frac"], 4),
                 "phase_ms_per_step": {k: round(v, 5) for k, v in r16["phases"].items()},
                 "error_vs_fp32_after_timed_steps": e16},
        "c2": {"workload": "drop sweeping particles 256x128x96, 20 spheres R=5, FP32",
               "steps": args.c2_steps, "mlups": round(r2["mlups"], 1),
               "ms_per_step": round(r2["ms_per_step"], 5),
               "roofline_frac": r2["roofline"]["frac"],
               "hbm_effective_frac": round(r2["hbm_effective_frac"], 4)},
        "c4": {"workload": "ensemble of 256 cubic boxes L in {48,64,80,96}, one sphere each, "
                           "FP32, graph replay",
               "runs_per_hour": round(c4["runs_per_hour"], 1), "run_steps": c4["run_steps"],
               "timed_steps": c4["steps"], "ms_per_step": round(c4["ms_per_step"], 4),
               "mlups": round(c4["mlups"], 1), "nodes": c4["nodes"]},
        "table1": {"workload": "the paper's drop-particle run: 400x181x71, R_p=10, drop R_d=50, "
                               "viscosity ratio 10 (drop tau 2.138, air 0.664), wall 100 deg, "
                               "particle 92 deg, Bo=1.25, FP32",
                   "steps": args.table1_steps, "mlups": round(rt1["mlups"], 1),
                   "ms_per_step": round(rt1["ms_per_step"], 5),
                   "roofline_frac": rt1["roofline"]["frac"]},
        "tube": {"workload": "sphere R_p=12.2 in pressure-driven flow through a tube R_t=40, "
                             "320x83x83, open ends (anti-bounce-back), tau 1.871, FP32",
                 "steps": args.tube_steps, "mlups": round(rtb["mlups"], 1),
                 "ms_per_step": round(rtb["ms_per_step"], 5),
                 "roofline_frac": rtb["roofline"]["frac"]},
        "textured": {"workload": "drop R=24 on a textured wall (8 pillars 12x12x8) with 6 spheres R=4, "
                                 "256x128x64, wall 110 deg, FP32",
                     "steps": args.textured_steps, "mlups": round(rtx["mlups"], 1),
                     "ms_per_step": round(rtx["ms_per_step"], 5),
                     "roofline_frac": rtx["roofline"]["frac"]},
    }
    if not args.no_cpu:
        c3_gpu = gpu_fields_after(c3w, args.cpu_steps)
        cb = cpu_baseline(c3w, args.cpu_steps, c3_gpu, c4)
        out["cpu_baseline"] = cb
        out["c4"]["error_gate"] = cb["ensemble_gate"]
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
