"""Throughput of the hybrid LB/FD step on one MI355X.

Default workload: the large single-GPU droplet-in-shear run, 1024 x 256 x 1024 nodes
(268M), two Shan-Chen components, Newtonian droplet R = 64, viscoelastic matrix (L^2 = 400,
De = 1), Ca = 0.2, FP32 populations (deviations from w rho0) and FP32 C - I, FP64
diagnostics every 100 steps.  Synthetic seeded inputs, resident in HBM before timing.

Prints one JSON line: MLUPS, ms/step, the HBM roofline of the step and the FP64 CPU
oracle timed on a bounded sub-box of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline (LBM+FENE-P step); FP32-vs-FP64 err; sweep time-to-D"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per node and step (FP32): populations read + written
# (2 x ncomp x 19 x 4) and C read + written (2 x 6 x 4)
ALG_BYTES = {1: 200, 2: 352}
# the Cholesky-log integrator also reads and writes its Adams-Bashforth history (2 x 6 x 4)
ALG_BYTES_AB2_HISTORY = 48
# kernels of one step per launch path (the chained step is the default)
STEP_KERNELS = {0: "k_fused (one launch per step)", 1: "k_moments + k_forces + k_collide",
                2: "k_moments + k_fused2 (two launches per step; bytes are the step's minimum)",
                3: "k_fused3 (one launch per step; it also forms the next step's moments)"}
LAUNCHES_PER_STEP = {0: 1, 1: 3, 2: 2, 3: 1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# committed counter summary per launch path (chained: k_fused3, two-pass: k_moments + k_fused2)
PROFILE_STEM = {2: "k_fused2", 3: "k_fused3"}


def recorded_traffic(workload, path_id, default_options=True):
    """HBM bytes per step (the step's launches together) on `workload`, from the committed
    rocprofv3 counter summary of that launch path (FETCH_SIZE and WRITE_SIZE, each scaled
    by what the counter reads for a copy of known size).  Returned only while the kernel
    sources hash to the profiled ones; a changed kernel gives None until it is profiled
    again.  The summaries profile the default options (BGK, upwind FENE-P): a run with
    other options gets None."""
    import hashlib

    if path_id not in PROFILE_STEM or not default_options:
        return None
    path = os.path.join(ROOT, "profiles",
                        f"{PROFILE_STEM[path_id]}_{workload.replace('droplet_shear_', 'droplet_')}.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic-record "):
            rec = json.loads(line[len("traffic-record "):])
    if not rec or rec.get("workload") != workload:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["sha256"]:
        return None
    rec["path"] = os.path.relpath(path, ROOT)
    return rec


def build_lattice(lb, workloads, nx, ny, nz, zchunk=16, collision="bgk", fene="upwind_euler", coupling="force",
                  kappa=0.0):
    """Create the droplet lattice and upload its fields slab by slab (host memory stays
    bounded for the 268M-node grid)."""
    wl0 = workloads.droplet_cfg2(nx=nx, ny=ny, nz=nz, box=(0, nx, 0, 1))
    wl0["params"]["collision"] = collision
    wl0["params"]["fene"] = fene
    wl0["params"]["coupling"] = coupling
    wl0["params"]["kappa"] = kappa
    lat = lb.Lattice(nx, ny, nz, 2, wl0["params"])
    lat.set_walls(wl0["walls"]["u_bottom"], wl0["walls"]["u_top"])
    for z0 in range(0, nz, zchunk):
        bz = min(zchunk, nz - z0)
        w = workloads.droplet_cfg2(nx=nx, ny=ny, nz=nz, box=(0, nx, z0, bz))
        lat.set_fields_box(0, 0, z0, nx, ny, bz, w["rho"], w["u"], w["C"])
    lat.reset_counters()
    return lat, wl0


def cpu_baseline(workloads, nx, ny, nz, budget_s=12.0, collision="bgk", fene="upwind_euler", keep=None,
                 coupling="force", kappa=0.0):
    """FP64 oracle on a 96 x ny x 96 sub-box window of the same workload (same per-node
    work), stepped until about `budget_s` seconds of CPU time have passed.  With `keep` (a
    dict), the window workload, the step count and the oracle's fields and diagnostics are
    left in it for the FP32-vs-FP64 comparison."""
    import oracle

    bx = min(96, nx)
    bz = min(96, nz)
    x0 = (nx - bx) // 2
    z0 = (nz - bz) // 2
    wl = workloads.droplet_cfg2(nx=nx, ny=ny, nz=nz, box=(x0, bx, z0, bz))
    wl["params"]["collision"] = collision
    wl["params"]["fene"] = fene
    wl["params"]["coupling"] = coupling
    wl["params"]["kappa"] = kappa
    o = oracle.from_workload(wl)
    nodes = bx * ny * bz
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 50:
            break
    if keep is not None:
        keep.update(wl=wl, steps=steps, fields=o.get_fields(), diag=o.diagnostics(),
                    desc=f"{bx}x{ny}x{bz} window at the centre of the {nx}x{ny}x{nz} droplet workload")
    cores = oracle.threads()
    # the same window on one thread, two steps (the oracle's results do not depend on it)
    oracle.set_threads(1)
    t1 = time.perf_counter()
    o.step(2)
    el1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    return {"value": nodes * steps / el / 1e6, "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} steps of a {bx}x{ny}x{bz} window of the same droplet workload "
                      f"({nodes} nodes, FP64, {el:.1f} s)",
            "cpu_model": cpu_model(),
            "one_thread_MLUPS": round(nodes * 2 / el1 / 1e6, 3),
            "one_thread_sample": f"2 further steps of the same window on 1 thread ({el1:.1f} s)"}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def sweep_judgement(plain, alt, paths, tol_d=0.01):
    """The answers of every sweep path against the plain per-case solves, and the fastest
    path whose answers are all within tol_d.

    plain: the per-case sweep on the library's default launch path, the chained step (the
    batched solve runs the same tile body, instance by instance bit for bit); alt: the
    per-case sweep on launch shapes autotuned per grid shape, a different rounding of the
    same steps.  Both are dicts with D, steady_step and wall_s.  paths: name -> (seconds, D
    per case) of the candidate paths.

    Every path is judged on every case the plain sweep brought to steady D, and only a path
    within tol_d on all of them qualifies.  Cases whose two plain answers differ by more
    than tol_d are reported as shape-sensitive (rounding decides their branch: a marginally
    stable droplet that stays or breaks up); that split is made from the two plain sweeps
    alone, and the scores over the remaining cases are reported beside the gating ones."""
    import numpy as np

    steady = np.asarray(plain["steady_step"]) > 0
    ref = np.asarray(plain["D"], dtype=np.float64)
    shape_sensitive = steady & (np.abs(np.asarray(alt["D"], dtype=np.float64) - ref) > tol_d)
    rest = steady & ~shape_sensitive

    def within(d, mask):
        return float(np.mean(np.abs(np.asarray(d, dtype=np.float64) - ref)[mask] <= tol_d)) if mask.any() else 1.0

    allp = dict(paths)
    allp["plain_tuned"] = (alt["wall_s"], alt["D"])
    gate = {k: within(d, steady) for k, (t, d) in allp.items()}
    cands = [(t, k) for k, (t, d) in allp.items() if gate[k] >= 1.0] + [(plain["wall_s"], "plain")]
    return {"steady": steady, "shape_sensitive": shape_sensitive, "best": min(cands),
            "within_all_steady": gate,
            "within_shape_insensitive": {k: within(d, rest) for k, (t, d) in allp.items()}}


def fp32_vs_fp64(lb, ref, path_id):
    """The GPU step (FP32, the launch path of the timed run) on the oracle's window, as
    many steps as the oracle ran, against the oracle's FP64 fields: relative L2 and max
    error of u, C and C - I, and the error of the deformation D."""
    import numpy as np

    lat = lb.from_workload(ref["wl"])
    lat.set_tuning(path_id, "32x8" if path_id in (lb.PATH_FUSED, lb.PATH_SPLIT) else "64x8", 0)
    lat.step(ref["steps"])
    g = lat.get_fields()
    dg = lat.diagnostics()
    lat.close()
    r = ref["fields"]
    eye = np.array([1, 1, 1, 0, 0, 0], dtype=np.float64)[:, None]

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    return {"window": ref["desc"], "steps": ref["steps"],
            "u_rel_l2": rel(g[1], r[1]), "u_max_abs": float(np.max(np.abs(g[1] - r[1]))),
            "u_max": float(np.max(np.abs(r[1]))),
            "C_rel_l2": rel(g[2], r[2]), "C_max_abs": float(np.max(np.abs(g[2] - r[2]))),
            "CmI_rel_l2": rel(g[2] - eye, r[2] - eye),
            "D_abs": abs(dg["D"] - ref["diag"]["D"]), "D": ref["diag"]["D"]}


def copy_probe(torch, gib, reps=20):
    """The library's streaming probe kernels (read, write, copy; plain and nontemporal
    stores; 16-byte accesses) over `gib` GiB buffers: the HBM rates a plain streaming kernel
    reaches on this part.  Then a plain device-to-device copy of `gib` GiB (bytes moved =
    2 x size per copy), whose FETCH_SIZE / WRITE_SIZE counters under rocprofv3 --pmc give the
    byte-counter scale."""
    import paper_1406_2686_amd as lb

    nbytes = int(gib * (1 << 30))
    rates = {}
    for kind in ("read", "write", "write_nt", "copy", "copy_nt"):
        r = lb.stream_probe(kind, nbytes, reps=reps)
        rates[kind] = {"ms": round(r["ms"], 4), "GB_per_s": round(r["GB_per_s"], 1),
                       "frac_of_peak": round(r["GB_per_s"] / HBM_PEAK_GBS, 4)}
    print(json.dumps({"stream_probe_GiB": gib, "kernels": rates}), flush=True)
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
    print(json.dumps({"copy_probe_GiB": gib, "bytes_per_copy": 2 * n * 4, "ms_per_copy": ms,
                      "GB_per_s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}),
          flush=True)


def sweep(lb, workloads, args):
    """Time to an answer within |dD| <= 0.01 of the plain steady D for a held-out set of
    droplet-in-shear cases.  Without the network: plain per-case solves (cold start, one
    lattice at a time) and one batched cold solve.  With it: two networks (different seeds)
    trained on batched solves of the training cases answer every held-out case; where they
    disagree by more than 0.005 in D the case falls back to a batched cold solve.  The plain
    solves judge every answer; `value` is the time of the fastest path whose answers are
    all within the tolerance."""
    import numpy as np

    from paper_1406_2686_amd import surrogate as sg

    # steady: D moved less than 1e-4 over each of two consecutive 1000-step windows (one
    # window is also met at slow extrema of a transient)
    crit = dict(every=100, window=1000, tol=1e-4, max_steps=args.max_steps, windows=2)
    if args.n_train == 0:
        return sweep_solver_only(lb, workloads, args, crit)
    train = workloads.sweep_cases(args.n_train, seed=4001, scale=args.scale)
    test = workloads.sweep_cases(args.n_test, seed=10001, scale=args.scale)
    wtrain = [workloads.sweep_workload(c) for c in train]
    wtest = [workloads.sweep_workload(c) for c in test]
    log(f"sweep: {len(train)} training / {len(test)} held-out cases, scale {args.scale}")
    gen = sg.solve(lb, wtrain, progress=log, **crit)
    ok = gen["steady_step"] > 0
    log(f"training data: {ok.sum()} steady of {len(train)} in {gen['wall_s']:.1f} s")
    X = sg.features(train)[ok]
    Y = np.stack([gen["D"], gen["theta"], gen["amp"]], 1)[ok]
    models = [sg.Surrogate(lb, seed=s, max_train=max(4096, len(train))) for s in (1, 2)]
    t0 = time.perf_counter()
    losses = [m.fit(X, Y, epochs=400, batch=128, lr=2e-3, seed=s + 10) for s, m in enumerate(models)]
    t_train = time.perf_counter() - t0
    plain = sg.solve_plain(lb, wtest, progress=log, tune="chained", **crit)
    log(f"plain sweep (chained path): {plain['wall_s']:.1f} s")
    alt = sg.solve_plain(lb, wtest, progress=log, tune="cached", **crit)
    log(f"plain sweep (shapes tuned per grid): {alt['wall_s']:.1f} s + tuning {alt['tuning_s']:.1f} s")
    cold = sg.solve(lb, wtest, progress=log, **crit)
    log(f"batched cold sweep: {cold['wall_s']:.1f} s")
    t0 = time.perf_counter()
    Xt = sg.features(test)
    p1, p2 = (m.predict(Xt) for m in models)
    pred = 0.5 * (p1 + p2)
    flag = np.abs(p1[:, 0] - p2[:, 0]) > 0.005
    t_pred = time.perf_counter() - t0
    answer = pred[:, 0].copy()
    t_fb = 0.0
    if flag.any():
        idx = np.nonzero(flag)[0]
        fb = sg.solve(lb, [wtest[i] for i in idx], progress=log, **crit)
        answer[idx] = fb["D"]
        t_fb = fb["wall_s"]
    log(f"surrogate + fallback: {flag.sum()} of {len(test)} solved, {t_pred + t_fb:.2f} s")
    # the surrogate's time counts its training data and training; the time without them
    # (both amortised over later sweeps) is printed beside it
    t_sur = gen["wall_s"] + t_train + t_pred + t_fb
    J = sweep_judgement(plain, alt, {"surrogate_with_fallback": (t_sur, answer),
                                     "surrogate_alone": (gen["wall_s"] + t_train + t_pred, pred[:, 0]),
                                     "batched_cold": (cold["wall_s"], cold["D"])})
    if args.save_data:
        np.savez(args.save_data, X_train=sg.features(train), Y_train=np.stack([gen["D"], gen["theta"], gen["amp"]], 1),
                 steady_train=gen["steady_step"], X_test=sg.features(test), D_plain=plain["D"], D_tuned=alt["D"],
                 steady_plain=plain["steady_step"], D_cold=cold["D"], pred1=p1, pred2=p2)
    steady = J["steady"]
    best = J["best"]
    out = {"metric": "sweep time-to-steady-D (|dD| <= 0.01 against plain solves)", "unit": "s",
           "value": round(best[0], 3), "path": best[1], "higher_is_better": False, "n_gpus": 1,
           "data": "synthetic", "dtype": "f32 solver, bf16 surrogate inference",
           "config": {"workload": f"droplet sweep, grids x{args.scale} of 64-192 x 32-64",
                      "n_train": len(train), "n_test": len(test), **crit},
           "plain_per_case_s": round(plain["wall_s"], 2), "plain_tuned_s": round(alt["wall_s"], 2),
           "plain_tuning_s": round(alt["tuning_s"], 2), "batched_cold_s": round(cold["wall_s"], 2),
           "batched_equals_plain": bool(np.array_equal(cold["D"], plain["D"])),
           "surrogate_end_to_end_s": round(t_sur, 2), "surrogate_amortised_s": round(t_pred + t_fb, 2),
           "surrogate_infer_s": round(t_pred, 4), "fallback_solve_s": round(t_fb, 2),
           "fallback_cases": int(flag.sum()), "training_data_s": round(gen["wall_s"], 2),
           "train_s": round(t_train, 2), "final_loss": losses,
           "steady_cases": int(steady.sum()), "shape_sensitive_cases": int(J["shape_sensitive"].sum()),
           "within_0.01_all_steady": J["within_all_steady"],
           "within_0.01_shape_insensitive": J["within_shape_insensitive"],
           "surrogate_mean_abs_dD": float(np.abs(pred[:, 0] - plain["D"])[steady].mean()),
           "unsteady_or_fault": {"plain": int((plain["steady_step"] <= 0).sum()),
                                 "cold": int((cold["steady_step"] <= 0).sum()),
                                 "training": int((~ok).sum())}}
    print(json.dumps(out), flush=True)


def sweep_solver_only(lb, workloads, args, crit):
    """The batched sweep without the network: the instances drawn with seed 3 (n_test of
    them, grids scaled by `scale`), solved to steady D once per case on its autotuned launch
    shape and once as one batch (chained body, captured graph), judged as in the sweep."""
    import numpy as np

    from paper_1406_2686_amd import surrogate as sg

    cases = workloads.sweep_cases(args.n_test, seed=3, scale=args.scale)
    wls = [workloads.sweep_workload(c) for c in cases]
    for w in wls:  # the schemes chosen on the command line (the paper's own, or the defaults)
        w["params"].update(collision=args.collision, fene=args.fene, coupling=args.coupling, kappa=args.kappa)
    nodes = [c["nx"] * c["ny"] * c["nz"] for c in cases]
    log(f"solver-only sweep: {len(cases)} cases, scale {args.scale}, {sum(nodes) / 1e6:.1f} M nodes")
    plain = sg.solve_plain(lb, wls, progress=log, tune="chained", **crit)
    log(f"plain sweep (chained path): {plain['wall_s']:.1f} s")
    alt = sg.solve_plain(lb, wls, progress=log, tune="cached", **crit)
    log(f"plain sweep (shapes tuned per grid): {alt['wall_s']:.1f} s + tuning {alt['tuning_s']:.1f} s")
    cold = sg.solve(lb, wls, progress=log, **crit)
    log(f"batched cold sweep: {cold['wall_s']:.1f} s")
    J = sweep_judgement(plain, alt, {"batched_cold": (cold["wall_s"], cold["D"])})
    steps_p = np.where(plain["steady_step"] > 0, plain["steady_step"], args.max_steps)
    fastest_plain = min(plain["wall_s"], alt["wall_s"])
    out = {"metric": "sweep time-to-steady-D (|dD| <= 0.01 against plain solves)", "unit": "s",
           "value": round(J["best"][0], 3), "path": J["best"][1], "higher_is_better": False, "n_gpus": 1,
           "data": "synthetic", "dtype": "f32",
           "config": {"workload": f"{len(cases)} droplet-in-shear instances (seed 3), grids x{args.scale} of "
                                  f"64-192 x 32-64", "nodes_total": int(sum(nodes)), "collision": args.collision,
                      "fene": args.fene, "coupling": args.coupling, "kappa": args.kappa, **crit},
           "plain_per_case_s": round(plain["wall_s"], 2), "plain_tuned_s": round(alt["wall_s"], 2),
           "plain_tuning_s": round(alt["tuning_s"], 2), "batched_cold_s": round(cold["wall_s"], 2),
           "batched_equals_plain": bool(np.array_equal(cold["D"], plain["D"])),
           "speedup_vs_fastest_plain": round(fastest_plain / cold["wall_s"], 2),
           "plain_MLUPS": round(float(np.dot(nodes, steps_p)) / plain["wall_s"] / 1e6, 1),
           "steady_cases": int(J["steady"].sum()), "shape_sensitive_cases": int(J["shape_sensitive"].sum()),
           "within_0.01_all_steady": J["within_all_steady"],
           "within_0.01_shape_insensitive": J["within_shape_insensitive"],
           "unsteady": {"plain": int((plain["steady_step"] == -1).sum()), "cold": int((cold["steady_step"] == -1).sum())},
           "fault": {"plain": int((plain["steady_step"] == -2).sum()), "cold": int((cold["steady_step"] == -2).sum())}}
    print(json.dumps(out), flush=True)


def batch_bench(lb, workloads, args):
    """Throughput of the batched step (one launch per step over every instance, replayed
    from the captured two-launch graph) on the droplet sweep family."""
    import torch

    cases = workloads.sweep_cases(args.batch, seed=4001, scale=args.scale)
    wls = [workloads.sweep_workload(c) for c in cases]
    # instances whose explicit polymer feedback goes unstable (fault flags) within the run
    # are screened out first: a faulting instance stops a plain batched step
    horizon = args.warmup + args.warmup % 2 + args.steps + args.steps % 2
    screen = lb.Batch(wls)
    _, ss = screen.run_to_steady(every=50, window=50 * (horizon // 50 + 2), tol=1e-300, max_steps=horizon + 50)
    screen.close()
    dropped = [i for i, s in enumerate(ss) if s == -2]
    wls = [w for i, w in enumerate(wls) if i not in dropped]
    nodes = sum(w["grid"]["nx"] * w["grid"]["ny"] * w["grid"]["nz"] for w in wls)
    b = lb.Batch(wls)
    if args.path == "chained":
        b.set_tuning(args.tile or "64x8", 0, path=lb.PATH_CHAINED)
    elif args.path == "fused":
        b.set_tuning("32x8", 0, path=lb.PATH_FUSED)
    elif args.path != "default":
        raise SystemExit("--batch runs the fused or the chained path")
    if args.path == "default" and args.tile:
        b.set_tuning(args.tile, 0, path=lb.PATH_CHAINED)
    tune = b.get_tuning()
    b.step(args.warmup + args.warmup % 2)
    torch.cuda.synchronize()
    K = args.steps + args.steps % 2
    a = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    a.record(b.stream)
    b.step(K)
    e.record(b.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = a.elapsed_time(e) / K
    achieved = ALG_BYTES[2] * nodes / (ms * 1e-3) / 1e9
    d = b.diagnostics()
    b.close()
    print(json.dumps({"metric": "batched step throughput (droplet sweep family)", "value": round(nodes * K / wall / 1e6, 1),
                      "unit": "MLUPS", "n_gpus": 1, "steps": K, "ms_per_step": round(ms, 4), "dtype": "f32",
                      "data": "synthetic", "higher_is_better": True,
                      "config": {"workload": f"{len(wls)} droplet-in-shear lattices, grids x{args.scale} of 64-192 x 32-64",
                                 "nodes": nodes, "faulting_instances_dropped": dropped,
                                 "launch": {"path": ["fused", "split", "two-pass", "chained"][tune["path"]],
                                            "tile": tune["tile"], "zchunk": tune["zchunk"]}},
                      "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                                   "kernel": ("k_fused3_batch" if tune["path"] == lb.PATH_CHAINED else "k_fused_batch")
                                   + " (all instances, one launch per step)"},
                      "fault_flags": int(max(x["flags"] for x in d))}), flush=True)


def mlp_bench(lb, workloads, args):
    """The surrogate network's kernels: BF16 inference on the matrix cores, FP32 forward,
    and on-device training (forward, backward, Adam per minibatch)."""
    import numpy as np
    import torch

    net = lb.MLP(max_batch=512, max_train=4096, seed=1)
    X, T = workloads.mlp_batch(4096, seed=5)
    Xi = X[:512]
    for _ in range(5):
        net.infer_bf16(Xi)
    reps = 200
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.infer_bf16(Xi)
    t_inf = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(Xi)
    t_fwd = (time.perf_counter() - t0) / reps
    epochs, batch = 50, 256
    t0 = time.perf_counter()
    loss = net.train(X, T, epochs=epochs, batch=batch, lr=2e-3, seed=3)
    t_train = time.perf_counter() - t0
    steps = epochs * (len(X) // batch)
    flop = 2 * (5 * 128 + 128 * 128 + 128 * 3)
    net.close()
    print(json.dumps({"metric": "surrogate network (5-128-128-3) kernels", "unit": "samples/s",
                      "value": round(512 / t_inf, 1), "n_gpus": 1, "dtype": "bf16 inference, f32 training",
                      "data": "synthetic", "higher_is_better": True,
                      "config": {"workload": "512-sample inference calls; 4096-sample training set, batch 256"},
                      "infer_bf16_call_ms": round(t_inf * 1e3, 4), "forward_f32_call_ms": round(t_fwd * 1e3, 4),
                      "train_step_ms": round(t_train / steps * 1e3, 4), "train_steps": steps,
                      "final_loss": loss, "flop_per_sample": flop}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--grid", type=str, default="1024x256x1024")
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--path", choices=["default", "chained", "two-pass", "fused", "split"], default="default",
                    help="launch path of the step (default: the library's, the chained step)")
    ap.add_argument("--collision", choices=["bgk", "mrt"], default="bgk",
                    help="collision operator (MRT runs on the split path)")
    ap.add_argument("--coupling", choices=["force", "stress"], default="force",
                    help="polymer stress as a body force (default) or in the equilibrium's second moment")
    ap.add_argument("--kappa", type=float, default=0.0,
                    help="artificial diffusivity of the Cholesky integrator (the paper gives no value)")
    ap.add_argument("--fene", choices=["upwind_euler", "cholesky_ab2"], default="upwind_euler",
                    help="FENE-P integrator (the Cholesky scheme runs on the split path)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="droplet-sweep mode: plain vs batched vs surrogate (with solver fallback) time to steady D")
    ap.add_argument("--n-train", type=int, default=2048)
    ap.add_argument("--n-test", type=int, default=256)
    ap.add_argument("--scale", type=float, default=0.5)
    ap.add_argument("--max-steps", type=int, default=12000)
    ap.add_argument("--save-data", default="",
                    help="sweep: write the training and held-out cases' features and solver answers (.npz)")
    ap.add_argument("--batch", type=int, default=0,
                    help="time the batched step over this many sweep lattices instead")
    ap.add_argument("--tile", choices=["64x8", "32x16"], default=None,
                    help="tile of the chained batch body (with --batch; default 64x8)")
    ap.add_argument("--mlp", action="store_true", help="time the surrogate network's kernels instead")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (HBM calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the multi-GPU (slab-decomposed) path is a design "
              "and is not implemented; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1406_2686_amd as lb
    import workloads

    if args.copy_probe > 0:
        copy_probe(torch, args.copy_probe)
        return
    if args.sweep:
        sweep(lb, workloads, args)
        return
    if args.batch > 0:
        batch_bench(lb, workloads, args)
        return
    if args.mlp:
        mlp_bench(lb, workloads, args)
        return

    nx, ny, nz = (int(v) for v in args.grid.split("x"))
    N = nx * ny * nz
    torch.cuda.set_device(0)
    t_init = time.perf_counter()
    lat, wl0 = build_lattice(lb, workloads, nx, ny, nz, collision=args.collision, fene=args.fene,
                             coupling=args.coupling, kappa=args.kappa)
    torch.cuda.synchronize()
    log(f"init {nx}x{ny}x{nz}: {time.perf_counter() - t_init:.1f} s")

    if args.path != "default":
        pid = {"fused": lb.PATH_FUSED, "split": lb.PATH_SPLIT, "two-pass": lb.PATH_TWOPASS,
               "chained": lb.PATH_CHAINED}[args.path]
        lat.set_tuning(pid, "32x8" if pid in (lb.PATH_FUSED, lb.PATH_SPLIT) else "64x8", 0)
    tuning = lat.get_tuning()
    d0 = lat.diagnostics()
    lat.step_async(args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done")

    stream = lat.stream
    K = args.steps
    every = max(1, args.diag_every)
    ev = []
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    done = 0
    diags = []
    while done < K:
        n = min(every, K - done)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lat.step_async(n)
        b.record(stream)
        ev.append((a, b, n))
        done += n
        if args.diag_every > 0:
            diags.append(lat.diagnostics())
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    step_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / K
    flags = lat.flags()
    d1 = lat.diagnostics()
    log(f"timed {K} steps: wall {wall:.2f} s, {step_ms:.3f} ms/step (events), flags={flags}")

    mlups = N * K / wall / 1e6
    alg_node = ALG_BYTES[2] + (ALG_BYTES_AB2_HISTORY if args.fene == "cholesky_ab2" else 0)
    alg = alg_node * N
    achieved = alg / (step_ms * 1e-3) / 1e9
    rec = recorded_traffic(f"droplet_shear_{nx}x{ny}x{nz}", tuning["path"],
                           args.collision == "bgk" and args.fene == "upwind_euler" and args.coupling == "force")
    traffic = None if rec is None else round(rec["bytes_per_step"] / (step_ms * 1e-3) / 1e9, 1)
    mass_drift = max(abs(d1["mass_A"] - d0["mass_A"]) / d0["mass_A"],
                     abs(d1["mass_B"] - d0["mass_B"]) / d0["mass_B"])
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / K, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"droplet_shear_{nx}x{ny}x{nz}", "nodes": N, "ncomp": 2,
                   "launch": {"path": ["fused", "split", "two-pass", "chained"][tuning["path"]], "tile": tuning["tile"],
                              "zchunk": tuning["zchunk"]},
                   "collision": args.collision, "fene": args.fene, "coupling": args.coupling, "kappa": args.kappa,
                   "droplet_R": wl0["meta"]["R"], "polymer": "matrix (L2=400, De=1)",
                   "diag_every": args.diag_every, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": STEP_KERNELS.get(tuning["path"], "?"),
                     "launches_per_step": LAUNCHES_PER_STEP[tuning["path"]],
                     "alg_bytes_per_node": alg_node, "event_ms_per_step": round(step_ms, 4),
                     "traffic_bytes_per_step": None if rec is None else rec["bytes_per_step"],
                     "traffic_source": None if rec is None else rec["path"]},
        "checks": {"fault_flags": flags, "mass_drift_rel": mass_drift, "D_final": d1["D"]},
    }
    lat.close()
    del lat
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        ref = {}
        out["cpu_baseline"] = cpu_baseline(workloads, nx, ny, nz, collision=args.collision, fene=args.fene, keep=ref,
                                           coupling=args.coupling, kappa=args.kappa)
        out["fp32_vs_fp64"] = fp32_vs_fp64(lb, ref, tuning["path"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
