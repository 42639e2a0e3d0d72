#!/usr/bin/env python3
"""Throughput of the AMR Euler hot path on one MI355X.

One step = one SSP-RK3 time step over every leaf patch of every level (CFL
time step, three stages of ghost fill + fused WENO5/Rusanov/divergence/RK
combine + coarse/fine flux correction + restriction), plus the gradient tag
and regrid every ``regrid_interval`` steps, on seeded synthetic data already
resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--config c2] [--exec batched|per_patch]
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


def flops_per_cell_stage(d: int, stage: int) -> int:
    """Algorithmic FP64 operations of one cell in one RK stage, counted on the
    definitions (add, mul, div, sqrt = 1; one edge and one face per cell and
    direction): primitives 3d+4; per direction 2(d+2) WENO5-JS evaluations of
    66 operations, two edge states of 4d+10, Rusanov 5(d+2), face flux
    5(d+2), divergence 3(d+2); the stage combination 2 (stage 1) or 5
    operations per variable."""
    nv = d + 2
    weno = 2 * nv * 66
    flux = 2 * (4 * d + 10) + 5 * nv
    per_dir = weno + flux + 5 * nv + 3 * nv
    combine = (2 if stage == 1 else 5) * nv
    return (3 * d + 4) + d * per_dir + combine


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


# largest base grid whose initial hierarchy the oracle steps within about a
# minute on one host core (2D 512^2)
ORACLE_MAX_BASE_CELLS = 1 << 18


def cpu_baseline(cfg, seed: int):
    """The oracle, as it stands, on a bounded sample: one SSP-RK3 step over the
    initial hierarchy of the same workload."""
    from paper_2508_05020_amd import workloads
    from oracle.solver import OracleAMR
    o = OracleAMR(cfg)
    o.init_from_ic(workloads.initial_data(cfg, seed))
    cells = o.leaf_cells()
    t0 = time.perf_counter()
    o.step()
    dt = time.perf_counter() - t0
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one SSP-RK3 step of the {cfg.name} initial hierarchy "
                      f"({cells} leaf cells, seed {seed}), numpy FP64, single thread, "
                      f"{dt:.1f} s"}


def copy_calibration() -> int:
    """10 copies of 1 GiB between two device buffers: a kernel whose HBM
    traffic is known (1 GiB read + 1 GiB written per launch)."""
    import torch
    n = 1 << 27  # float64 elements = 1 GiB
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


def learned_gain(args) -> int:
    """Train the refinement predictor on the solver's own tags, then compare
    regridding policies on one seeded run (2D quadrants + blobs, or 3D blast
    waves + density perturbations): wall-clock per unit simulated time, judge
    failures (fallbacks), regrids and cell updates.  Every policy runs under
    the plain-tag judge with fallback, so all advance on meshes that cover the
    plain tags at the same rate."""
    import numpy as np
    from paper_2508_05020_amd import amr, learned, workloads

    H, b, dim = args.learned_every, args.learned_buffer, args.learned_dim
    seed_eval = args.seed_eval if args.seed_eval is not None else (4100 if dim == 2 else 5100)
    rounds = args.learned_rounds if args.learned_rounds is not None else (1 if dim == 2 else 2)
    if dim == 2:
        # the patch edge of the evaluation workload when one is named (the 2D
        # network predicts leaves of one edge), else 16
        n = 16
        if args.learned_eval:
            edges = set(workloads.config(args.learned_eval).patch_cells)
            if len(edges) != 1:
                raise SystemExit("the 2D network needs one patch edge on every level")
            n = edges.pop()
        cfg = workloads.AMRConfig(name="quadrants-blobs-4lev", dim=2, base_cells=max(64, 2 * n),
                                  patch_cells=[n] * 4, periodic=[True, True],
                                  ic="quadrants_blobs", tag_buffer=b, max_patches=16384)
        seeds = list(range(4000, 4000 + args.train_runs))
        stride = 2
    else:
        n = 8
        cfg = workloads.AMRConfig(name="blasts-perturbed-4lev", dim=3, base_cells=16,
                                  patch_cells=[n] * 4, periodic=[True] * 3,
                                  ic="blasts_perturbed", tag_buffer=b, max_patches=32768)
        seeds = list(range(5000, 5000 + args.train_runs))
        stride = 4
    res = tuple(cfg.base_cells * 2 ** l for l in range(cfg.max_levels))
    t0 = time.perf_counter()
    mean, std = learned.input_statistics(
        [learned.uniform_config(cfg.base_cells, n, tag_buffer=b, dim=dim)], seeds[:1], steps=8)
    data = learned.build_dataset(res, seeds, steps=40, horizon=H, stride=stride, mean=mean,
                                 std=std, n=n, tag_buffer=b, dim=dim)
    val = learned.build_dataset(res[-2:], [seed_eval], steps=40, horizon=H, stride=4,
                                mean=mean, std=std, n=n, tag_buffer=b, dim=dim)
    pos = float(data.y.mean())
    pos_weight = float(min(100.0, (1.0 - pos) / max(pos, 1e-6)))
    log(f"[learned] {data.x.shape[0]} training tiles from {len(seeds)} runs at {res}, "
        f"positive cells {pos:.3f} ({time.perf_counter() - t0:.1f} s)")

    # evaluation workload: the training configuration, or a named one (its
    # dilation set to the one the labels were made with)
    ecfg, eseed = cfg, seed_eval
    if args.learned_eval:
        ecfg = workloads.config(args.learned_eval).replace(tag_buffer=b)
        if ecfg.dim != dim:
            raise SystemExit(f"--learned-eval {args.learned_eval} is {ecfg.dim}D, the network {dim}D")
        num = args.learned_eval[1:] if args.learned_eval[1:].isdigit() else "0"
        eseed = workloads.seed_for(int(num), 1)

    def hier(mode=amr.EXEC_BATCHED, c=None, seed=None):
        c = ecfg if c is None else c
        h = amr.Hierarchy(c, exec_mode=mode)
        amr.init_from_ic(h, workloads.initial_data(c, eseed if seed is None else seed))
        return h

    if not args.learned_eval:
        h = hier()
        learned.run_policy(h, 8, 2, "plain", judge=True)  # warm-up outside the comparison
        h.close()
    h_bl = hier() if not args.learned_eval else hier(c=cfg, seed=seed_eval)
    pred = amr.Predictor(h_bl, n, mean, std, pos_weight=pos_weight, max_batch=256)
    pred.set_weights(learned.init_weights(seed=1, dim=dim))
    t1 = time.perf_counter()
    losses = learned.train(pred, data, epochs=args.epochs, lr=2e-3, batch=64)
    train_s = time.perf_counter() - t1
    tau = learned.choose_tau(pred, val, recall=0.99)
    met = learned.patch_metrics(pred, val, tau)
    pred.predict(0, tau)  # first use of the inference kernels, outside the comparison
    log(f"[learned] trained in {train_s:.1f} s, loss {losses[0]:.3f} -> {losses[-1]:.3f}, "
        f"tau {tau:.4f}, validation {met}")

    if args.learned_eval:
        # the evaluation hierarchy gets its own predictor with the trained
        # weights; one large hierarchy at a time
        weights = pred.get_weights()
        pred.close()
        h_bl.close()
        import torch
        torch.cuda.empty_cache()

    results = {}
    steps = args.steps
    for name, every, policy, mode in (("plain2_per_patch", 2, "plain", amr.EXEC_PER_PATCH),
                                      ("plain2", 2, "plain", amr.EXEC_BATCHED),
                                      (f"plain{H}", H, "plain", amr.EXEC_BATCHED),
                                      (f"learned{H}", H, "learned", amr.EXEC_BATCHED)):
        if args.learned_eval and mode == amr.EXEC_PER_PATCH:
            continue  # one launch per patch and phase: hours on a large workload
        if policy == "learned" and args.learned_eval:
            h = hier()
            pred = amr.Predictor(h, n, mean, std, pos_weight=pos_weight, max_batch=256)
            pred.set_weights(weights)
            pred.predict(0, tau)
        else:
            h = h_bl if policy == "learned" else hier(mode)
        st = learned.run_policy(h, steps, every, policy, pred if policy == "learned" else None,
                                tau, judge=True, rounds=rounds)
        results[name] = st.as_dict()
        log(f"[learned] {name}: {results[name]}")
        if policy != "learned":
            h.close()
            if args.learned_eval:
                import torch
                torch.cuda.empty_cache()
    L = results[f"learned{H}"]["wall_per_tsim"]
    desc = (f"{ecfg.name}: {dim}D base {ecfg.base_cells}^{dim}, {ecfg.max_levels} levels of "
            f"{ecfg.patch_cells} patches, dilation {b}, seed {eseed}, {steps} steps")
    if args.learned_eval:
        desc += (f"; network trained on {cfg.name} ({dim}D base {cfg.base_cells}^{dim}, "
                 f"{n}^{dim} patches)")
    out = {"metric": "wall-clock per unit simulated time, plain vs learned regridding",
           "config": {"workload": desc},
           "learned_rounds": rounds,
           "training": {"tiles": int(data.x.shape[0]), "runs": len(seeds), "horizon": H,
                        "epochs": args.epochs, "first_loss": losses[0], "final_loss": losses[-1],
                        "seconds": train_s, "tau": tau, "validation": met},
           "policies": results,
           "gain_vs_plain2_per_patch": (results["plain2_per_patch"]["wall_per_tsim"] / L
                                        if "plain2_per_patch" in results else None),
           "gain_vs_plain2": results["plain2"]["wall_per_tsim"] / L,
           f"gain_vs_plain{H}": results[f"plain{H}"]["wall_per_tsim"] / L}
    print(json.dumps(out), flush=True)
    pred.close()
    return 0


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
                         "500 for c2; 128 for --learned; 50 calls for --diag)")
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--seed", type=int, default=None,
                    help="initial-data seed (default: 1000 * config number + 1)")
    ap.add_argument("--exec", dest="exec_mode", default="batched", choices=["batched", "per_patch"])
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
    ap.add_argument("--learned-every", type=int, default=16,
                    help="regrid interval of the learned policy (and forecast horizon)")
    ap.add_argument("--learned-buffer", type=int, default=1, help="tag dilation in cells")
    ap.add_argument("--diag", action="store_true",
                    help="time the velocity-gradient diagnostic instead of the step")
    ap.add_argument("--learned-rounds", type=int, default=None,
                    help="predict + regrid rounds per learned regrid (each can add one level; "
                         "default 1 in 2D, 2 in 3D)")
    ap.add_argument("--learned-eval", default=None,
                    help="evaluate the policies on this workload (e.g. c5) instead of the "
                         "training configuration; per-patch launches are skipped there")
    ap.add_argument("--learned-dim", type=int, default=2, choices=[2, 3],
                    help="2D quadrants + blobs or 3D blast waves + perturbations")
    ap.add_argument("--seed-eval", type=int, default=None,
                    help="seed of the evaluation run (default 4100 in 2D, 5100 in 3D)")
    ap.add_argument("--train-runs", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (scales HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
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
    if args.steps is None:
        args.steps = cfg.steps
    if args.seed is None:
        num = args.config[1:] if args.config[:1] == "c" and args.config[1:].isdigit() else "2"
        args.seed = workloads.seed_for(int(num), 1)
    mode = amr.EXEC_BATCHED if args.exec_mode == "batched" else amr.EXEC_PER_PATCH
    h = amr.Hierarchy(cfg, exec_mode=mode)
    amr.init_from_ic(h, workloads.initial_data(cfg, args.seed))
    log(f"[bench] {cfg.name}: initial hierarchy {h.counts()} patches (active, leaf), "
        f"{h.leaf_cells()} leaf cells")
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
        per = {}
        for g in (False, True):
            h.set_graph(g)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            advance(16, False)
            torch.cuda.synchronize()
            per[g] = (time.perf_counter() - t0) / 16
        use_graph = per[True] < per[False]
        log(f"[bench] step graph {per[True] * 1e6:.0f} us, eager {per[False] * 1e6:.0f} us: "
            f"{'graph' if use_graph else 'eager'}")
    h.set_graph(use_graph and mode == amr.EXEC_BATCHED)
    # pass 1: whole-job throughput (step graphs replayed, no instrumentation)
    t0 = time.perf_counter()
    cells = advance(args.steps, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s")
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
    f_step = sum(flops_per_cell_stage(d, s) for s in (1, 2, 3))
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
            "step_graph": bool(use_graph and mode == amr.EXEC_BATCHED),
            "tile": None if tile is None else {"variant": tile[0], "extent": tile[1],
                                               "threads": tile[2],
                                               "xy_edges_in_one_sweep": tile[0] >= 8},
            "leaf_cells_per_step_avg": cells / max(1, args.steps),
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_stage (fused WENO5-JS + Rusanov + Eq. (9) divergence + RK combine)",
            "achieved": achieved_tf,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tf / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic(None if tile is None else tile[0], cells_per_launch),
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
    if not args.no_cpu_baseline:
        if cfg.base_cells ** cfg.dim > ORACLE_MAX_BASE_CELLS:
            # one oracle step over this initial hierarchy would take hours
            out["cpu_baseline"] = None
            log(f"[bench] no cpu_baseline: {cfg.base_cells}^{cfg.dim} base cells is beyond the "
                f"oracle's bounded sample ({ORACLE_MAX_BASE_CELLS})")
        else:
            log("[bench] timing the oracle on a bounded sample")
            out["cpu_baseline"] = cpu_baseline(cfg, args.seed)
    print(json.dumps(out), flush=True)
    h.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
