#!/usr/bin/env python3
"""Throughput of the AMR Euler hot path on one MI355X.

One step = one SSP-RK3 time step over every leaf patch of every level (CFL
time step, three stages of ghost fill + fused WENO5/Rusanov/divergence/RK
combine + coarse/fine flux correction + restriction), plus the gradient tag
and regrid every ``regrid_interval`` steps, on seeded synthetic data already
resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--config c5] [--exec batched|per_patch]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "FP64 cell-updates/s (all levels) + % HBM roofline; batched+learned vs plain"
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X dense FP64 vector
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E


def flops_per_cell_stage(d: int, stage: int, scheme: str = "weno") -> int:
    """Algorithmic FP64 operations of one cell in one RK stage, counted on the
    definitions (add, mul, div, sqrt = 1; one edge and one face per cell and
    direction).  WENO5-JS on primitives: primitives 3d+4; per direction
    2(d+2) WENO5-JS evaluations of 66 operations, two edge states of 4d+10,
    Rusanov 5(d+2), face flux 5(d+2), divergence 3(d+2); the stage
    combination 2 (stage 1) or 5 operations per variable.  Central (Eq. 8):
    the interpolations are 4 operations and one value serves both sides.
    Characteristic variables: no primitives; per direction the mean state
    2(d+2), its eigensystem 3d+14, six node projections of 4d+9, 2(d+2)
    WENO5-JS evaluations, two back projections of 4d+10, two positivity
    tests of 3d+4, two conserved-state fluxes with signal speed of 4d+12,
    then Rusanov, face flux and divergence as above."""
    nv = d + 2
    tail = 5 * nv + 5 * nv + 3 * nv
    if scheme == "char":
        per_dir = (2 * nv + (3 * d + 14) + 6 * (4 * d + 9) + 2 * nv * 66 + 2 * (4 * d + 10)
                   + 2 * (3 * d + 4) + 2 * (4 * d + 12) + tail)
        prim = 0
    else:
        interp = nv * 4 if scheme == "central" else 2 * nv * 66
        per_dir = interp + 2 * (4 * d + 10) + tail
        prim = 3 * d + 4
    combine = (2 if stage == 1 else 5) * nv
    return prim + d * per_dir + combine


def bytes_per_cell_stage(d: int, stage: int) -> int:
    """Algorithmic HBM bytes of one cell in one stage: read U^n (and the stage
    input at stages 2-3), write the output; FP64, d+2 variables."""
    return (2 if stage == 1 else 3) * (d + 2) * 8


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


ROOT = os.path.dirname(os.path.abspath(__file__))
COUNTERS = os.path.join(ROOT, "profiles", "k_stage_counters.json")
# sources the stage kernel is compiled from
KERNEL_SOURCES = ("paper_2508_05020_amd/csrc/stage.hip", "paper_2508_05020_amd/csrc/device_common.hpp",
                  "paper_2508_05020_amd/csrc/amr_internal.hpp")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(variant, cells_per_launch):
    """HBM bytes per stage-kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the copy-kernel
    calibration, per leaf cell of the launch), or None when the summary is
    missing, was taken on another kernel source, or on another tile variant."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if variant is None or c.get("source_sha256") != kernel_source_hash():
        return None
    v = c.get("variants", {}).get(str(variant))
    if not v:
        return None
    return (v["fetch_bytes_per_cell"] + v["write_bytes_per_cell"]) * cells_per_launch


# largest 2D base grid whose initial hierarchy the oracle steps within about a
# minute on one host core (512^2)
ORACLE_MAX_BASE_CELLS = 1 << 18


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown CPU"


def cpu_baseline(cfg, seed: int, scheme: str = "weno"):
    """The oracle, as it stands, on a bounded sample of the workload: one
    SSP-RK3 step over a hierarchy it builds itself from the same generator
    and seed.  In 3D the sample is the benchmark layout (patches 32/16/16/8,
    4 levels) on a 64^3 base, refined around the first blast so that every
    level has coarse/fine faces (about 750 k leaf cells); in 1D and 2D it
    is the workload's own initial hierarchy.  numpy, one thread."""
    from paper_2508_05020_amd import workloads
    from oracle.solver import OracleAMR
    gen = workloads.initial_data(cfg, seed)
    if cfg.dim == 3:
        sc = workloads.c5_sample_config().replace(ic=cfg.ic, cfl=cfg.cfl, gamma=cfg.gamma)
        o = OracleAMR(sc, scheme=scheme)
        for k in o.forest.keys():
            o.set_initial(k, gen)
        for keys in workloads.blast_refinements(sc, seed):
            o.regrid(keys, [], gen)
        what = (f"one SSP-RK3 step of the oracle on the {cfg.name} layout (patches "
                f"{sc.patch_cells}, {sc.max_levels} levels) over a {sc.base_cells}^3 base "
                f"refined around the first blast of the same generator ({cfg.ic}, seed {seed})")
    elif cfg.base_cells ** cfg.dim <= ORACLE_MAX_BASE_CELLS:
        o = OracleAMR(cfg, scheme=scheme)
        o.init_from_ic(gen)
        what = f"one SSP-RK3 step of the oracle over the {cfg.name} initial hierarchy (seed {seed})"
    else:
        return None
    cells = o.leaf_cells()
    t0 = time.perf_counter()
    o.step()
    dt = time.perf_counter() - t0
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}: {cells} leaf cells in {dt:.1f} s; numpy FP64, single thread, "
                      f"{host_cpu()}"}


def _counter_csv(path: str, kernel: str, counter: str):
    """Per-dispatch values of one counter for the kernels whose name contains
    `kernel`, in dispatch order, from a rocprofv3 counter_collection CSV."""
    import csv
    vals = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter:
                d = int(r["Dispatch_Id"])
                vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
    return [vals[d] for d in sorted(vals)]


def ingest_counters(args) -> int:
    """Write profiles/k_stage_counters.json from rocprofv3 counter runs: the
    stage kernel's FETCH_SIZE and WRITE_SIZE per dispatch (KiB) on a run of
    `bench.py --no-autotune --tile T` whose first steps do not regrid (every
    dispatch covers the log's leaf cells), scaled by what the same counters
    read for device copies of known size."""
    import re
    d = args.ingest_counters
    tile = args.tile
    with open(os.path.join(d, "s_fetch.log")) as f:
        log_text = f.read()
    cells = int(re.search(r"stage kernel: \d+ launches over \d+ steps, [\d.]+ ms, (\d+) leaf cells",
                          log_text).group(1))
    workload = re.search(r"\[bench\] (\S+): initial hierarchy", log_text).group(1)
    gib = args.copy_gib
    cal_f = _counter_csv(os.path.join(d, "cal_fetch", "run_counter_collection.csv"),
                         "copyBuffer", "FETCH_SIZE")
    cal_w = _counter_csv(os.path.join(d, "cal_write", "run_counter_collection.csv"),
                         "copyBuffer", "WRITE_SIZE")
    copy_kib = gib * 1024 * 1024
    sf = copy_kib / (sum(cal_f) / len(cal_f))
    sw = copy_kib / (sum(cal_w) / len(cal_w))
    fetch = _counter_csv(os.path.join(d, "s_fetch", "run_counter_collection.csv"), "k_stage",
                         "FETCH_SIZE")
    write = _counter_csv(os.path.join(d, "s_write", "run_counter_collection.csv"), "k_stage",
                         "WRITE_SIZE")
    rec = {"kernel": "k_stage", "workload": workload, "leaf_cells_per_dispatch": cells,
           "dispatches": len(fetch), "source_sha256": kernel_source_hash(),
           "scale": {"fetch": sf, "write": sw, "copy_gib": gib},
           "variants": {str(tile): {
               "fetch_bytes_per_cell": sum(fetch) / len(fetch) * 1024 * sf / cells,
               "write_bytes_per_cell": sum(write) / len(write) * 1024 * sw / cells,
               "fetch_bytes_per_cell_by_stage": [
                   sum(fetch[k::3]) / len(fetch[k::3]) * 1024 * sf / cells for k in range(3)],
               "write_bytes_per_cell_by_stage": [
                   sum(write[k::3]) / len(write[k::3]) * 1024 * sw / cells for k in range(3)]}},
           "commands": "see k_stage_c5.md"}
    with open(COUNTERS, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))
    return 0


def copy_calibration(gib: int = 1) -> int:
    """10 copies of ``gib`` GiB between two device buffers: a kernel whose
    HBM traffic is known (gib GiB read + gib GiB written per launch)."""
    import torch
    n = gib << 27  # float64 elements
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_bytes_per_launch": 2 * 8 * n, "launches": 10,
                      "GBps": 10 * 2 * 8 * n / dt / 1e9}), flush=True)
    return 0


def train_predictor(dim: int, horizon: int, buffer: int, runs: int, epochs: int,
                    recall: float, seed_eval: int, base: int, n: int = None, res=None):
    """Train the refinement predictor on the solver's own tags: single-level
    periodic runs of the workload's generator (2D quadrants + blobs on 16^2
    patches, 3D blasts + perturbations on 8^3 tiles) at resolutions ``res``
    (default base and 2 base), seeds 4000 + k (2D) or 5000 + k (3D), labels
    = the plain tagger's dilated tags over the next ``horizon`` steps.
    Returns the trained weights and what the comparison needs
    (normalisation, tau for ``recall`` of the held-out patches)."""
    from paper_2508_05020_amd import amr, learned, workloads
    if n is None:
        n = 16 if dim == 2 else 8
    seeds = list(range(4000 if dim == 2 else 5000, (4000 if dim == 2 else 5000) + runs))
    res = tuple(res) if res else (base, 2 * base)
    t0 = time.perf_counter()
    mean, std = learned.input_statistics(
        [learned.uniform_config(base, n, tag_buffer=buffer, dim=dim)], seeds[:1], steps=8)
    data = learned.build_dataset(res, seeds, steps=32, horizon=horizon, stride=4, mean=mean,
                                 std=std, n=n, tag_buffer=buffer, dim=dim)
    val = learned.build_dataset(res, [seed_eval], steps=32, horizon=horizon, stride=4,
                                mean=mean, std=std, n=n, tag_buffer=buffer, dim=dim)
    data_s = time.perf_counter() - t0
    pos = float(data.y.mean())
    pos_weight = float(min(100.0, (1.0 - pos) / max(pos, 1e-6)))
    log(f"[learned] {data.x.shape[0]} training tiles from {len(seeds)} runs at {res}, "
        f"positive cells {pos:.3f} ({data_s:.1f} s)")
    cfg = learned.uniform_config(base, n, tag_buffer=buffer, dim=dim)
    h = amr.Hierarchy(cfg)
    pred = amr.Predictor(h, n, mean, std, pos_weight=pos_weight, max_batch=256)
    pred.set_weights(learned.init_weights(seed=1, dim=dim))
    t1 = time.perf_counter()
    losses = learned.train(pred, data, epochs=epochs, lr=2e-3, batch=64)
    train_s = time.perf_counter() - t1
    tau = learned.choose_tau(pred, val, recall=recall)
    met = learned.patch_metrics(pred, val, tau)
    weights = pred.get_weights()
    pred.close()
    h.close()
    log(f"[learned] trained in {train_s:.1f} s, loss {losses[0]:.3f} -> {losses[-1]:.3f}, "
        f"tau {tau:.4f}, validation {met}")
    return {"n": n, "mean": mean, "std": std, "pos_weight": pos_weight, "tau": tau,
            "weights": weights,
            "info": {"tiles": int(data.x.shape[0]), "runs": len(seeds),
                     "resolutions": list(res), "horizon": horizon, "epochs": epochs,
                     "first_loss": losses[0], "final_loss": losses[-1],
                     "data_seconds": data_s, "train_seconds": train_s, "tau": tau,
                     "recall_target": recall, "validation": met}}


def compare_policies(ecfg, eseed: int, steps: int, policies, trained, rounds: int):
    """Wall-clock per unit simulated time of regridding policies on one
    workload, each from its own fresh initial hierarchy, all under the
    plain-tag judge with fallback (every step covers the plain tags at the
    workload's own dilation).  ``policies``: (name, every, kind, exec mode,
    regrid dilation or None)."""
    import torch
    from paper_2508_05020_amd import amr, learned, workloads
    results = {}
    for name, every, kind, mode, buf in policies:
        t0 = time.perf_counter()
        h = amr.Hierarchy(ecfg, exec_mode=mode)
        amr.init_from_ic(h, workloads.initial_data(ecfg, eseed))
        pred = None
        if kind == "learned":
            pred = amr.Predictor(h, trained["n"], trained["mean"], trained["std"],
                                 pos_weight=trained["pos_weight"], max_batch=256)
            pred.set_weights(trained["weights"])
            pred.predict(0, trained["tau"])  # first use of the kernels, outside the timing
        torch.cuda.synchronize()
        log(f"[learned] {name}: initial hierarchy in {time.perf_counter() - t0:.1f} s")
        st = learned.run_policy(h, steps, every, kind, pred, trained["tau"] if pred else 0.5,
                                judge=True, rounds=rounds, regrid_buffer=buf, progress=8)
        results[name] = st.as_dict()
        log(f"[learned] {name}: {results[name]}")
        if pred is not None:
            pred.close()
        h.close()
        del h
        torch.cuda.empty_cache()
    return results


def learned_gain(args) -> int:
    """Train the refinement predictor on the solver's own tags, then compare
    regridding policies on one seeded run: wall-clock per unit simulated
    time, judge fallbacks, regrids, cell updates and coverage."""
    import math
    from paper_2508_05020_amd import amr, workloads
    H, b, dim = args.learned_every, args.learned_buffer, args.learned_dim
    seed_eval = args.seed_eval if args.seed_eval is not None else (4100 if dim == 2 else 5100)
    rounds = args.learned_rounds if args.learned_rounds is not None else (1 if dim == 2 else 2)
    n = None
    if dim == 2 and args.learned_eval:
        # the 2D network predicts leaves of one patch edge
        edges = set(workloads.config(args.learned_eval).patch_cells)
        if len(edges) != 1:
            raise SystemExit("the 2D network needs one patch edge on every level")
        n = edges.pop()
    trained = train_predictor(dim, H, b, args.train_runs, args.epochs, args.recall, seed_eval,
                              base=64 if dim == 2 else 32, n=n, res=args.train_res)
    if args.learned_eval:
        ecfg = workloads.config(args.learned_eval).replace(tag_buffer=b)
        if ecfg.dim != dim:
            raise SystemExit(f"--learned-eval {args.learned_eval} is {ecfg.dim}D, the network {dim}D")
        num = args.learned_eval[1:] if args.learned_eval[1:].isdigit() else "0"
        eseed = workloads.seed_for(int(num), 1)
    else:
        n = trained["n"]
        base = args.learned_base or (64 if dim == 2 else 16)
        ecfg = workloads.AMRConfig(
            name=f"{'quadrants-blobs' if dim == 2 else 'blasts-perturbed'}-4lev", dim=dim,
            base_cells=base, patch_cells=[n] * 4, periodic=[True] * dim,
            ic="quadrants_blobs" if dim == 2 else "blasts_perturbed", tag_buffer=b,
            max_patches=(16384 * max(1, (base // 64) ** 2) if dim == 2
                         else 32768 * max(1, (base // 16) ** 3 // 2)))
        eseed = seed_eval
    wide = min(3, math.ceil(H * ecfg.cfl))
    policies = [("P_plain2_per_patch", 2, "plain", amr.EXEC_PER_PATCH, None),
                ("B_plain2", 2, "plain", amr.EXEC_BATCHED, None),
                (f"B{H}_plain{H}_dilation{wide}", H, "plain", amr.EXEC_BATCHED, wide),
                (f"BL_learned{H}", H, "learned", amr.EXEC_BATCHED, None)]
    if (args.learned_eval and dim == 3) or args.learned_base:
        policies = policies[1:]  # one launch per patch and phase: hours on a large workload
    results = compare_policies(ecfg, eseed, args.steps, policies, trained, rounds)
    L = results[f"BL_learned{H}"]["wall_per_tsim"]
    out = {"metric": "wall-clock per unit simulated time, plain vs learned regridding",
           "config": {"workload": f"{ecfg.name}: {dim}D base {ecfg.base_cells}^{dim}, "
                                  f"{ecfg.max_levels} levels of {ecfg.patch_cells} patches, "
                                  f"dilation {b}, seed {eseed}, {args.steps} steps"},
           "learned_rounds": rounds, "training": trained["info"], "policies": results,
           "gain_vs": {k: v["wall_per_tsim"] / L for k, v in results.items()}}
    print(json.dumps(out), flush=True)
    return 0


def learned_vs_plain(cfg, args):
    """The metric's third part on the benchmark workload itself: the
    predictor trained on the generator's own tags, then batched plain
    regridding every 2 steps (B), batched plain regridding at the workload's
    interval with the dilation widened to ceil(interval x CFL) (at most 3,
    B8), and batched learned regridding at that interval (BL), each for
    ``--learned-steps`` steps from a fresh initial hierarchy under the
    plain-tag judge, so that every policy runs at the same (full) coverage
    of the plain tags.  The per-patch policy is not run on this workload (one
    launch per patch and phase)."""
    import math
    from paper_2508_05020_amd import amr
    H = cfg.regrid_interval
    t0 = time.perf_counter()
    if cfg.dim == 2 and len(set(cfg.patch_cells)) != 1:
        return None  # the 2D network predicts leaves of one patch edge
    trained = train_predictor(cfg.dim, H, cfg.tag_buffer, args.train_runs, args.epochs,
                              args.recall, 5100 if cfg.dim == 3 else 4100,
                              base=64 if cfg.dim == 3 else 128,
                              n=8 if cfg.dim == 3 else cfg.patch_cells[0],
                              res=(64,) if cfg.dim == 3 else None)
    wide = min(3, math.ceil(H * cfg.cfl))
    policies = [("B_plain2", 2, "plain", amr.EXEC_BATCHED, None),
                (f"B{H}_plain{H}_dilation{wide}", H, "plain", amr.EXEC_BATCHED, wide),
                (f"BL_learned{H}", H, "learned", amr.EXEC_BATCHED, None)]
    res = compare_policies(cfg, args.seed, args.learned_steps, policies, trained,
                           rounds=2 if cfg.dim == 3 else 1)
    L = res[f"BL_learned{H}"]["wall_per_tsim"]
    return {"unit": "s wall per unit simulated time", "steps": args.learned_steps,
            "policies": {k: {"wall_per_tsim": v["wall_per_tsim"], "coverage": v["coverage"],
                             "regrids": v["regrids"], "fallbacks": v["fallbacks"],
                             "capacity_retries": v["capacity_retries"],
                             "cell_updates": v["cell_updates"], "t_sim": v["t_sim"]}
                         for k, v in res.items()},
            "learned_speedup_vs": {k: v["wall_per_tsim"] / L for k, v in res.items()},
            "training": trained["info"],
            "seconds": time.perf_counter() - t0}


def diag_bench(args) -> int:
    """Time the velocity-gradient diagnostic (ghost fill of the leaves plus
    the gradient kernel) on a workload's hierarchy after a few steps."""
    import torch
    from paper_2508_05020_amd import amr, workloads
    cfg = workloads.config(args.config)
    seed = args.seed
    if seed is None:
        num = args.config[1:] if args.config[:1] == "c" and args.config[1:].isdigit() else "2"
        seed = workloads.seed_for(int(num), 1)
    h = amr.Hierarchy(cfg)
    amr.init_from_ic(h, workloads.initial_data(cfg, seed))
    for _ in range(4):
        h.step()
    d = cfg.dim
    out = torch.empty((d * d + 1, h.state_doubles // h.nvar), dtype=torch.float64, device=h.device)
    for _ in range(args.warmup):
        h.velocity_gradient(0, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(h.stream)
    for _ in range(args.steps):
        h.velocity_gradient(0, out)
    e1.record(h.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    cells = h.leaf_cells()
    # algorithmic bytes per leaf cell: (d + 1) values read, d*d + 1 written
    b_cell = 8 * ((d + 1) + (d * d + 1))
    print(json.dumps({"metric": "velocity-gradient diagnostic (fill + kernel) per call",
                      "config": {"workload": cfg.name, "leaf_cells": cells},
                      "ms_per_call": ms, "calls": args.steps,
                      "bytes_per_cell": b_cell,
                      "GBps_whole_call": cells * b_cell / ms / 1e6}), flush=True)
    h.close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's configured run length, "
                         "200 for c5; 128 for --learned; 50 calls for --diag)")
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--base", type=int, default=None,
                    help="level-0 cells per dimension instead of the workload's (a smaller "
                         "hierarchy of the same layout and generator)")
    ap.add_argument("--seed", type=int, default=None,
                    help="initial-data seed (default: 1000 * config number + 1)")
    ap.add_argument("--exec", dest="exec_mode", default="batched", choices=["batched", "per_patch"])
    ap.add_argument("--scheme", default="weno", choices=["weno", "central", "char"],
                    help="edge interpolation: WENO5-JS of the primitives (default), the central "
                         "interpolation of Eq. (8), or WENO5-JS of characteristic variables")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--step-graph", choices=["auto", "on", "off"], default="auto",
                    help="replay each step as a hipGraph, launch eagerly, or time both "
                         "(16 steps each, regrids included, after the warm-up) and keep the "
                         "faster")
    ap.add_argument("--tile", type=int, default=None,
                    help="use this stage-kernel tile variant instead of autotuning")
    ap.add_argument("--learned", action="store_true",
                    help="train the refinement predictor and compare regrid policies")
    ap.add_argument("--learned-every", type=int, default=8,
                    help="regrid interval of the learned policy (and forecast horizon)")
    ap.add_argument("--learned-buffer", type=int, default=2, help="tag dilation in cells")
    ap.add_argument("--diag", action="store_true",
                    help="time the velocity-gradient diagnostic instead of the step")
    ap.add_argument("--learned-rounds", type=int, default=None,
                    help="predict + regrid rounds per learned regrid (each can add one level; "
                         "default 1 in 2D, 2 in 3D)")
    ap.add_argument("--learned-eval", default=None,
                    help="evaluate the policies on this workload (e.g. c5) instead of the "
                         "training configuration; per-patch launches are skipped there")
    ap.add_argument("--learned-base", type=int, default=None,
                    help="level-0 cells per dimension of the evaluation hierarchy of --learned "
                         "(default 64 in 2D, 16 in 3D)")
    ap.add_argument("--learned-dim", type=int, default=2, choices=[2, 3],
                    help="2D quadrants + blobs or 3D blast waves + perturbations")
    ap.add_argument("--seed-eval", type=int, default=None,
                    help="seed of the evaluation run (default 4100 in 2D, 5100 in 3D)")
    ap.add_argument("--train-runs", type=int, default=16,
                    help="seeded single-level runs the predictor is trained on")
    ap.add_argument("--train-res", type=int, nargs="+", default=None,
                    help="resolutions of the single-level training runs (default: the "
                         "training base and twice it)")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--recall", type=float, default=0.995,
                    help="fraction of held-out patches with a future tag the mask must flag")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-versus-plain regridding comparison of the default run")
    ap.add_argument("--learned-steps", type=int, default=24,
                    help="steps per policy in the default run's regridding comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (scales HBM counters)")
    ap.add_argument("--copy-gib", type=int, default=1, help="size of each calibration copy")
    ap.add_argument("--ingest-counters", default=None, metavar="DIR",
                    help="write profiles/k_stage_counters.json from rocprofv3 counter runs in "
                         "DIR (s_fetch/, s_write/, cal_fetch/, cal_write/ and s_fetch.log; "
                         "--tile names the profiled variant)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_gib)
    if args.ingest_counters:
        return ingest_counters(args)
    if args.learned:
        if args.steps is None:
            args.steps = 128
        return learned_gain(args)
    if args.diag:
        if args.steps is None:
            args.steps = 50
        return diag_bench(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is described in the design notes, not built.",
              file=sys.stderr)
        return 2

    import torch
    from paper_2508_05020_amd import amr, workloads

    cfg = workloads.config(args.config)
    if args.base is not None:
        cfg = cfg.replace(name=f"{cfg.name}-base{args.base}", base_cells=args.base)
        cfg.validate()
    if args.steps is None:
        args.steps = cfg.steps
    if args.seed is None:
        num = args.config[1:] if args.config[:1] == "c" and args.config[1:].isdigit() else "2"
        args.seed = workloads.seed_for(int(num), 1)
    mode = amr.EXEC_BATCHED if args.exec_mode == "batched" else amr.EXEC_PER_PATCH
    scheme = {"weno": amr.SCHEME_WENO, "central": amr.SCHEME_CENTRAL,
              "char": amr.SCHEME_CHAR}[args.scheme]
    t_init = time.perf_counter()
    h = amr.Hierarchy(cfg, exec_mode=mode, scheme=scheme)
    amr.init_from_ic(h, workloads.initial_data(cfg, args.seed))
    log(f"[bench] {cfg.name}: initial hierarchy {h.counts()} patches (active, leaf), "
        f"{h.leaf_cells()} leaf cells ({time.perf_counter() - t_init:.1f} s)")
    tile = None
    if args.tile is not None:
        h.set_tile_variant(args.tile)
        tile = h.tile_variant()
        log(f"[bench] tile variant {tile}")
    elif mode == amr.EXEC_BATCHED and not args.no_autotune:
        best, best_ms = h.autotune(5)
        tile = h.tile_variant()
        log(f"[bench] autotuned tile variant {tile} ({best_ms * 1e3:.1f} us per RHS launch)")
    else:
        tile = h.tile_variant()

    nstep = 0

    def advance(k: int, count: bool):
        nonlocal nstep
        cells = 0
        for _ in range(k):
            if count:
                cells += h.leaf_cells()
            h.step()
            nstep += 1
            if cfg.regrid_interval > 0 and nstep % cfg.regrid_interval == 0:
                h.adapt()
        return cells

    advance(args.warmup, False)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")
    use_graph = args.step_graph == "on"
    if mode == amr.EXEC_BATCHED and args.step_graph == "auto":
        # throughput (leaf cell-updates per second) rather than time per step:
        # the mesh, and with it the work per step, changes between the windows
        per, rate = {}, {}
        for g in (False, True):
            h.set_graph(g)
            advance(2, False)  # records the two step graphs (one per rate slot)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c = advance(16, True)
            torch.cuda.synchronize()
            per[g] = (time.perf_counter() - t0) / 16
            rate[g] = c / (16 * per[g])
        use_graph = rate[True] > rate[False]
        log(f"[bench] step graph {per[True] * 1e6:.0f} us ({rate[True] / 1e9:.3f} G cell-updates/s), "
            f"eager {per[False] * 1e6:.0f} us ({rate[False] / 1e9:.3f} G): "
            f"{'graph' if use_graph else 'eager'}")
    h.set_graph(use_graph and mode == amr.EXEC_BATCHED)
    # pass 1: whole-job throughput (step graphs replayed, no instrumentation)
    rec0 = h.graph_records()
    regrids0 = nstep
    t0 = time.perf_counter()
    cells = advance(args.steps, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    rec_timed = h.graph_records() - rec0
    regrids_timed = (nstep // cfg.regrid_interval - regrids0 // cfg.regrid_interval
                     if cfg.regrid_interval > 0 else 0)
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s ({regrids_timed} regrids, "
        f"{rec_timed} step graphs recorded)")
    # pass 2: the fused stage kernel timed with HIP events around every launch
    # (eager launches on the same stream; kernel work is identical)
    psteps = min(args.steps, args.profile_steps)
    h.profile(True)
    pcells = advance(psteps, True)
    torch.cuda.synchronize()
    ms, launches, kcells = h.profile_read()
    h.profile(False)
    cells_per_launch = kcells / max(1, launches)
    log(f"[bench] stage kernel: {launches} launches over {psteps} steps, {ms:.2f} ms, "
        f"{cells_per_launch:.0f} leaf cells per launch")
    if h.check() != 0:
        log("[bench] WARNING: non-physical cells after the run")
    d = cfg.dim
    f_step = sum(flops_per_cell_stage(d, s, args.scheme) for s in (1, 2, 3))
    b_step = sum(bytes_per_cell_stage(d, s) for s in (1, 2, 3))
    # every timed step launches the stage kernel once per stage over all leaf
    # cells (batched) or once per tile group (per-patch): totals per step
    total_flops = pcells * f_step
    total_bytes = pcells * b_step
    kern_s = ms * 1e-3
    achieved_tf = total_flops / kern_s / 1e12 if kern_s > 0 else 0.0
    achieved_gbs = total_bytes / kern_s / 1e9 if kern_s > 0 else 0.0
    value = cells / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / max(1, args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: {d}D Euler gamma={cfg.gamma}, base {cfg.base_cells}^{d}, "
                        f"{cfg.max_levels} levels, patches {cfg.patch_cells}, "
                        f"{'periodic' if all(cfg.periodic) else 'mixed bc'}, ic {cfg.ic} "
                        f"seed {args.seed}, CFL {cfg.cfl}, regrid every {cfg.regrid_interval}",
            "exec": args.exec_mode,
            "scheme": args.scheme,
            "step_graph": bool(use_graph and mode == amr.EXEC_BATCHED),
            "regrids_timed": regrids_timed,
            "step_graphs_recorded_timed": rec_timed,
            "tile": None if tile is None else {"variant": tile[0], "extent": tile[1],
                                               "threads": tile[2],
                                               "xy_edges_in_one_sweep": tile[0] >= 8},
            "leaf_cells_per_step_avg": cells / max(1, args.steps),
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_stage (fused " + {"weno": "WENO5-JS of the primitives",
                                           "central": "central interpolation (Eq. (8))",
                                           "char": "WENO5-JS of characteristic variables"}[
                args.scheme] + " + Rusanov + Eq. (9) divergence + RK combine)",
            "achieved": achieved_tf,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tf / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic(None if tile is None or args.scheme != "weno" else tile[0],
                                        cells_per_launch),
            "launches": launches,
            "avg_launch_ms": ms / max(1, launches),
            "cells_per_launch": cells_per_launch,
            "flops_per_cell_update": f_step,
        },
        "roofline_hbm": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "bytes_per_cell_update": b_step,
            "whole_step_frac": cells * b_step / elapsed / 1e9 / HBM_PEAK_GBS,
        },
    }
    h.close()
    del h
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(cfg, args.seed, args.scheme)
        if out["cpu_baseline"] is None:
            log(f"[bench] no cpu_baseline: {cfg.base_cells}^{cfg.dim} base cells is beyond the "
                f"oracle's bounded sample")
    if not args.no_learned and mode == amr.EXEC_BATCHED and cfg.dim >= 2 \
            and cfg.regrid_interval > 2 and args.scheme == "weno":
        out["learned_vs_plain"] = learned_vs_plain(cfg, args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
