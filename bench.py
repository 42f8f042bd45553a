#!/usr/bin/env python3
"""Benchmark of the batched FP64 FMM interaction kernels on one MI355X.

Workload (default): 32^3 = 32768 sub-grids (256^3 = 16.8M cells) of a
synthetic two-blob binary-star field (blob widths in {2h, 4h}, mass ratio
drawn from U[0.3, 1.0]), periodic, 20% of the sub-grids missing 1..9
neighbours. A step is the whole hot path over that batch: the batched
multipole forward and its adjoint (source-role and target-role passes),
replayed as one captured hipGraph. Inputs are resident in HBM before the
timed region.

Metric: FP64 cell-pair interactions per second of forward+backward; the pair
count is exact (from the neighbour table). Also reported: the roofline of the
dominant kernel (algorithmic FLOPs per launch / mean launch time, measured
with HIP events on the launch stream), forward-only throughput, the batched
launch against per-sub-grid launches of the single-block kernel on the
4096-sub-grid forward workload (1, 8 and 32 streams), and the CPU oracle on a
bounded sample of the same workload.

Progress goes to stderr; stdout gets one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("FP64 cell-pair interactions/s (fwd, fwd+bwd): batched vs per-subgrid launch, "
          "% FP64 peak")
PEAK_FP64_TFLOPS = 78.6  # 256 CUs x 128 FP64 FLOP/clk x 2.4 GHz

# Method-level FP64 operations per cell pair (FMA = 2, rsqrt = 1), the basis of
# every roofline fraction of the interaction: the forward (derivatives of 1/r
# to order 3 and the 84-FMA contraction) 224; the adjoint (derivatives to order
# 4, 84 FMA for the moment gradient, 84 + 60 FMA for the position-gradient
# summand, which serves the target and the source of a pair alike) 556; the
# step 780.
METHOD_FLOP = {"forward": 224, "adjoint": 556, "step": 780}

# Per-launch counts of this implementation (secondary): the plain formulas
# each kernel evaluates -- derivatives of 1/r to order 3 (incl. r = X_i - X_j):
# 61, to order 4: 121; forward contraction 84 FMA; adjoint source-role pass
# 84 + 111 FMA; target-role pass 64 + 111 FMA. The two adjoint passes each
# evaluate the order-4 derivatives and the position-gradient terms, so their
# sum (982) exceeds the method's 556.
FLOP_PER_PAIR = {
    "forward": 61 + 2 * 84,                # 229
    "adjoint_source": 121 + 2 * (84 + 111),  # 511
    "adjoint_target": 121 + 2 * (64 + 111),  # 471
    # the two-launch step: the forward that saves the target-side sums
    # evaluates the order-4 derivatives, the forward contraction (84 FMA) and
    # the order-4 terms of orders 1..4 (111 FMA); the one-pass adjoint is the
    # source-role pass (its per-cell epilogue adds the target role)
    "forward_save": 121 + 2 * (84 + 111),    # 511
    "adjoint_saved": 121 + 2 * (84 + 111),   # 511
    # the forward with the angular-momentum correction: the same pair loop as
    # the forward with saved sums (a per-cell epilogue contracts the order-4
    # sums with the target's moments)
    "forward_amc": 121 + 2 * (84 + 111),     # 511
}


def sched_name(s):
    """Name of a one-pass schedule code (shape, optionally + persistent)."""
    base = {1: "W8", 2: "W16", 3: "W8P2"}[s & 0xF]
    return base + ("+persistent" if s & 0x10 else "") + ("+xcd-local" if s & 0x20 else "")

# sources of the interaction kernels (the counter record names their hash)
INTERACTION_SOURCES = ("ot_common.h", "ot_interact.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_counters(kernel, sched, n):
    """Counter record of this kernel and schedule from the committed rocprofv3
    summary (HBM-side bytes per launch: FETCH_SIZE + WRITE_SIZE scaled by a
    plain copy of known size; issued FP64 operations per launch from the F64
    instruction counters), when it was taken on these interaction sources and
    this workload; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_32768_subgrids.json")
    if n != 32 or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in INTERACTION_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2303_08058_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != rec.get("source_sha256_16"):
        return None
    if kernel == "adjoint_source":
        sched = sched >> 8
    elif kernel == "adjoint_target":
        sched = sched & 0xff
    key = (kernel + {1: "_w8", 2: "_w16", 3: "_w8p2"}[sched & 0xF] + ("_persistent" if sched & 0x10 else "")
           + ("_local" if sched & 0x20 else ""))
    return rec["kernels"].get(key)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32, help="sub-grids per axis (32: 256^3 cells)")
    ap.add_argument("--per-subgrid-n", type=int, default=16,
                    help="sub-grids per axis of the batched-vs-per-sub-grid comparison (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time of the oracle baseline (0: skip)")
    ap.add_argument("--tree-steps", type=int, default=10,
                    help="timed launches of each tree pass (0: skip)")
    ap.add_argument("--full-steps", type=int, default=2,
                    help="timed launches of the full-truncation forward (0: skip)")
    ap.add_argument("--full-sched", type=lambda v: int(v, 0), default=None,
                    help="schedule of the full-truncation forward (default: fastest of the library default W8P2+persistent+xcd-local, W8 and W8P2)")
    ap.add_argument("--no-two-level", action="store_true",
                    help="skip the two-level step (its parent-level forward shares the forward kernel)")
    ap.add_argument("--fwd-sched", type=lambda v: int(v, 0), default=None,
                    help="forward schedule code (skips the autotuner; e.g. 0x22 = W16 + XCD-local order)")
    ap.add_argument("--bwd-sched", type=lambda v: int(v, 0), default=None,
                    help="backward schedule code, target role | source role << 8 (with --fwd-sched)")
    ap.add_argument("--save-sched", type=lambda v: [int(x, 0) for x in v.split(",")], default=None,
                    help="schedules of the two-launch step, forward,adjoint (skips its autotuner; e.g. 0x33,0x33)")
    ap.add_argument("--no-two-pass", action="store_true",
                    help="skip the three-launch step (plain forward, two adjoint passes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU only (sharding the sub-grids over GPUs "
              "is a design note, not implemented). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2303_08058_amd as ot
    import synthetic

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    # ------------------------------------------------------------------ inputs
    t0 = time.time()
    batch, M, X = synthetic.config5(args.n)
    log("inputs: %d sub-grids generated in %.1f s" % (batch["S"], time.time() - t0))
    plan = ot.Plan.from_batch(batch)
    pairs = plan.pairs()
    w = synthetic.weights(batch["T"], 2005)
    Md, Xd, wd = d(M), d(X), d(w)
    NS, NT = batch["S"] * 512, batch["T"] * 512
    L = torch.empty((20, NT), dtype=torch.float64, device=dev)
    gM = torch.empty((20, NS), dtype=torch.float64, device=dev)
    gX = torch.empty((3, NS), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    log("plan: %d targets, %d pairs" % (batch["T"], pairs))

    def time_step():
        for _ in range(args.warmup):
            plan.step_graph_launch()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        e0.record(stream)
        for i in range(args.steps):
            plan.step_graph_launch()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        return e0.elapsed_time(e1) / args.steps, wall * 1e3 / args.steps

    def kernel_stats(kt):
        out = {}
        for k, (ms, n) in kt.items():
            if n == 0:
                continue
            mean = ms / n
            out[k] = {"mean_ms": round(mean, 4), "launches": n,
                      "impl_tflops": round(pairs * FLOP_PER_PAIR[k] / (mean * 1e-3) / 1e12, 3),
                      "impl_flop_per_pair": FLOP_PER_PAIR[k]}
            log("kernel %-15s %.3f ms  %.2f TFLOP/s (implementation count)" % (k, mean, out[k]["impl_tflops"]))
        return out

    kernels = {}
    two_pass = None
    fs = bs = None
    if not args.no_two_pass:
        # three-launch step: plain forward, source- and target-role adjoint passes
        if args.fwd_sched is not None and args.bwd_sched is not None:
            fs, bs = args.fwd_sched, args.bwd_sched
        else:
            fs, bs = plan.autotune(Md, Xd, L, wd, gM, gX)
        log("three-launch step: forward %s, adjoint target role %s, source role %s"
            % (sched_name(fs), sched_name(bs & 0xff), sched_name(bs >> 8)))
        plan.step_graph_create(Md, Xd, L, wd, gM, gX, fs, bs)
        ms_two, wall_two = time_step()
        log("three-launch graph step: %.2f ms (wall %.2f ms)" % (ms_two, wall_two))
        plan.set_timing(True)
        plan.kernel_times()
        for i in range(args.steps):
            plan.multipole_batched(Md, Xd, L, sched=fs)
            plan.multipole_backward(Md, Xd, wd, gM, gX, sched=bs)
        kernels.update(kernel_stats(plan.kernel_times()))
        plan.set_timing(False)
        adj2_ms = kernels["adjoint_source"]["mean_ms"] + kernels["adjoint_target"]["mean_ms"]
        two_pass = {
            "ms_per_step": round(ms_two, 3), "pairs_per_s": pairs / (ms_two * 1e-3),
            "schedules": {"forward": sched_name(fs), "adjoint_target": sched_name(bs & 0xff),
                          "adjoint_source": sched_name(bs >> 8)},
            "fwd_bwd_frac_fp64_peak": round(pairs * METHOD_FLOP["step"] / (ms_two * 1e-3) / 1e12
                                            / PEAK_FP64_TFLOPS, 4),
            "adjoint_ms": round(adj2_ms, 3),
            "adjoint_frac_fp64_peak": round(pairs * METHOD_FLOP["adjoint"] / (adj2_ms * 1e-3) / 1e12
                                            / PEAK_FP64_TFLOPS, 4),
        }

    # two-launch step (the timed step): the forward that saves the target-side
    # sums, and the one-pass adjoint that uses them
    Cs = torch.empty((ot.NSAVED, NT), dtype=torch.float64, device=dev)
    if args.save_sched is not None:
        sf, sb = args.save_sched
    else:
        sf, sb = plan.autotune_saved(Md, Xd, L, Cs, wd, gM, gX)
    log("two-launch step: forward with saved sums %s, one-pass adjoint %s" % (sched_name(sf), sched_name(sb)))
    plan.step_graph_create_saved(Md, Xd, L, Cs, wd, gM, gX, sf, sb)
    ms_per_step, wall_step = time_step()
    log("two-launch graph step: %.2f ms (wall %.2f ms)" % (ms_per_step, wall_step))
    plan.set_timing(True)
    plan.kernel_times()
    for i in range(args.steps):
        plan.multipole_batched_save(Md, Xd, L, Cs, sched=sf)
        plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX, sched=sb)
    kernels.update(kernel_stats(plan.kernel_times()))
    plan.set_timing(False)
    del Cs
    # the forward with the angular-momentum correction of the force (not part
    # of the step), with the forward-with-saved-sums schedule
    dF = torch.empty((3, NT), dtype=torch.float64, device=dev)
    plan.multipole_batched_amc(Md, Xd, L, dF, sched=sf)
    plan.set_timing(True)
    plan.kernel_times()
    for i in range(args.steps):
        plan.multipole_batched_amc(Md, Xd, L, dF, sched=sf)
    kernels.update(kernel_stats(plan.kernel_times()))
    plan.set_timing(False)
    del dF
    if fs is None:
        fs = sf  # forward schedule of the two-level step (W8 / W8P2 also serve the plain forward)
    # roofline: the step's two launches together, at the method's 780 FLOP per
    # pair (the forward's 224 and the adjoint's 556): the forward launch does
    # part of the adjoint's work, so neither launch alone has a method count
    step_kern_ms = kernels["forward_save"]["mean_ms"] + kernels["adjoint_saved"]["mean_ms"]
    achieved = round(pairs * METHOD_FLOP["step"] / (step_kern_ms * 1e-3) / 1e12, 3)
    dom = max(("forward_save", "adjoint_saved"), key=lambda k: kernels[k]["mean_ms"])
    counters = measured_counters(dom, sf if dom == "forward_save" else sb, args.n)
    traffic = None if counters is None else counters["fetch_bytes"] + counters["write_bytes"]
    issued = None if counters is None else round(
        counters["issued_fp64_flop"] / (kernels[dom]["mean_ms"] * 1e-3) / 1e12, 3)
    fwd_pairs_s = fwd_tflops = None
    if "forward" in kernels:
        fwd_pairs_s = pairs / (kernels["forward"]["mean_ms"] * 1e-3)
        fwd_tflops = pairs * METHOD_FLOP["forward"] / (kernels["forward"]["mean_ms"] * 1e-3) / 1e12
    sum_ms = step_kern_ms
    fwdbwd_flops = pairs * METHOD_FLOP["step"] / (ms_per_step * 1e-3) / 1e12

    # copy of known size, for scaling HBM counters (not part of the step)
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float64, device=dev)  # 2 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # ----------------------------------------- tree passes on the same store
    tree = None
    if args.tree_steps > 0 and args.n % 2 == 0:
        tree = tree_passes(args.n, args.tree_steps, Md, Xd, L, ot, synthetic, np, torch, dev,
                           plan=plan, batch=batch)

    # ------------------------------------ forward with the full truncation
    full = None
    if args.full_steps > 0:
        full = full_truncation(plan, pairs, args.full_steps, Md, Xd, L, ot, torch, args.full_sched,
                               wd, gM, gX)

    # ------------------------------------------------- a two-level FMM step
    two_level = None
    if args.tree_steps > 0 and args.n % 2 == 0 and not args.no_two_level:
        two_level = two_level_step(args.n, args.tree_steps, plan, batch, fs, Md, Xd, L, ot, synthetic,
                                   np, torch, dev)
        if args.full_steps > 0:
            two_level["full_truncation"] = two_level_step(args.n, args.full_steps, plan, batch, fs, Md, Xd,
                                                          L, ot, synthetic, np, torch, dev, full=True)

    # --------------------------------------- batched vs per-sub-grid launches
    per_sub = None
    if args.per_subgrid_n > 0:
        per_sub = per_subgrid_comparison(args.per_subgrid_n, ot, synthetic, np, torch, dev)

    # ----------------------------------------------------------- CPU oracle
    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(batch, M, X, w, args.cpu_seconds, np)

    out = {
        "metric": METRIC,
        "value": pairs / (ms_per_step * 1e-3),
        "unit": "cell-pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "batched multipole forward+adjoint, %d^3 sub-grids (%d^3 cells), "
                        "periodic, 20%% of sub-grids missing 1-9 neighbours, hipGraph step"
                        % (args.n, 8 * args.n),
            "subgrids": batch["S"], "cells": batch["S"] * 512, "pairs": pairs,
            "field": batch["field"],
            "schedules": {"forward_save": sched_name(sf), "adjoint_saved": sched_name(sb)},
            "step": "forward with saved target-side sums + one-pass adjoint (two launches)",
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu", "kernel": "the step's two launches (forward with saved sums + one-pass adjoint)",
            "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
            "traffic_kernel": dom,
            "traffic_unit": "bytes per launch of the longer of the two launches (HBM side, FETCH_SIZE + "
                            "WRITE_SIZE, copy-calibrated)",
            "flop_basis": "method-level FP64 ops per cell pair of forward + adjoint, 780 (FMA = 2, rsqrt = 1) "
                          "x exact pairs, over the summed mean durations of the two launches",
            "issued_fp64_tflops": issued,
            "issued_basis": "FP64 operations per launch of the longer launch counted by rocprofv3 "
                            "(64 x (2 FMA + MUL + ADD + TRANS) instruction counters, committed summary) "
                            "/ its live mean duration",
        },
        "kernels": kernels,
        "method_flop_per_pair": METHOD_FLOP,
        "three_launch_step": two_pass,
        "fwd_tflops": None if fwd_tflops is None else round(fwd_tflops, 3),
        "fwd_frac_fp64_peak": None if fwd_tflops is None else round(fwd_tflops / PEAK_FP64_TFLOPS, 4),
        "fwd_bwd_tflops": round(fwdbwd_flops, 3),
        "fwd_bwd_frac_fp64_peak": round(fwdbwd_flops / PEAK_FP64_TFLOPS, 4),
        "fwd_pairs_per_s": fwd_pairs_s,
        "direct_launch_ms_per_step": round(sum_ms, 3),
        "tree_passes": tree,
        "two_level_step": two_level,
        "full_truncation": full,
        "batched_vs_per_subgrid": per_sub,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# Algorithmic HBM bytes of the tree passes (FP64, every input read once and
# every output written once):
#   upward pass, per parent cell: 8 children x (20 moments + 3 centre) read,
#     20 moments + 3 centre written                          -> 1656 B
#   downward pass, per child cell: parent's 20 + 3 read once per 8 children,
#     child centre (3) read, child coefficients (20) read and written -> 367 B
#   evaluation, per cell: 20 moments + 20 coefficients read, 3 force
#     components + 1 energy written                          -> 352 B
TREE_BYTES = {"m2m": 1656, "l2l": 367, "evaluate": 352}
PEAK_HBM_GBS = 8000.0


def tree_passes(n, steps, Md, Xd, L, ot, synthetic, np, torch, dev, plan=None, batch=None):
    """Times the upward pass from the n^3 store to its (n/2)^3 parent level,
    the downward pass back into the store's coefficients, the local
    evaluation over every cell and, with a plan, the coarse substitutes of
    its missing neighbours (taken from the parent level the upward pass
    wrote); HIP events on the launch stream."""
    ch = synthetic.octree_children(n)
    Sp, S = ch.shape[0], n ** 3
    tree = ot.Tree(ch, S)
    f64 = dict(dtype=torch.float64, device=dev)
    Mp = torch.empty((20, Sp * 512), **f64)
    Xp = torch.empty((3, Sp * 512), **f64)
    Lp = torch.randn((20, Sp * 512), generator=torch.Generator(device=dev).manual_seed(7), **f64)
    F = torch.empty((3, S * 512), **f64)
    W = torch.empty((S * 512,), **f64)
    stream = torch.cuda.current_stream()
    calls = {
        "m2m": (lambda: tree.m2m(Md, Xd, Mp, Xp), Sp * 512),
        "l2l": (lambda: tree.l2l(Lp, Xp, Xd, L), S * 512),
        "evaluate": (lambda: ot.ot_fmm_evaluate(Md, L, F, W), S * 512),
    }
    out = {}
    for name, (fn, units) in calls.items():
        for _ in range(2):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        gbs = TREE_BYTES[name] * units / (ms * 1e-3) / 1e9
        out[name] = {"mean_ms": round(ms, 4), "units": units, "unit": "parent cell" if name == "m2m"
                     else "cell", "bytes_per_unit": TREE_BYTES[name],
                     "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                                  "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)}}
        log("tree %-9s %.3f ms  %.0f GB/s" % (name, ms, gbs))
    tree.close()
    if plan is not None:
        coarse, octant = synthetic.coarse_tables(n, batch)
        cpairs = plan.set_coarse(Sp, coarse, octant)
        ntg = int((coarse >= 0).any(1).sum())
        # both truncations; the full one counted like the full forward
        for key, full, fpp in (("coarse_fine", False, FLOP_PER_PAIR["forward"]),
                               ("coarse_fine_full", True, FULL_FLOP_REDUCED)):
            for _ in range(2):
                plan.coarse_fine(Xd, Mp, Xp, L, full=full)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(steps):
                plan.coarse_fine(Xd, Mp, Xp, L, full=full)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            tf = cpairs * fpp / (ms * 1e-3) / 1e12
            out[key] = {
                "mean_ms": round(ms, 4), "targets": ntg, "substituted_slots": int((coarse >= 0).sum()),
                "pairs": cpairs, "unit": "(target cell, coarse cell) pair", "flop_per_pair": fpp,
                "roofline": {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_TFLOPS, 4)}}
            log("%-16s %.3f ms  %d targets, %d pairs, %.2f TFLOP/s" % (key, ms, ntg, cpairs, tf))
    # a plain device copy of 2 GiB on the same stream, as the attainable
    # read+write bandwidth these streaming kernels compare with
    a = torch.empty(1 << 28, **f64)
    b = torch.empty_like(a)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    out["copy_2GiB"] = {"mean_ms": round(ms, 4),
                        "gbs": round(2 * a.numel() * 8 / (ms * 1e-3) / 1e9, 1)}
    log("copy 2 GiB      %.3f ms  %.0f GB/s" % (ms, out["copy_2GiB"]["gbs"]))
    del a, b
    return out


# FP64 operations per cell pair of the full-truncation forward (every output
# |a| <= 3 keeps every moment |b| <= 3; derivatives to order 6):
#   as the kernel evaluates it -- r, 1/r and the radial factors D_0..D_6: 21;
#   the derivative recursion over the 64 derivatives the trace-reduced
#   contraction reads: 223; 16 x 16 reduced products: 512           -> 756
#   plain formulas -- all 84 derivatives by the same recursion (443 + 21) and
#   all 20 x 20 products (800)                                       -> 1264
# The plain count overstates the executed work by 1.67x (its rate would pass
# the hardware peak), so the roofline uses the reduced count.
FULL_FLOP_REDUCED = 756
FULL_FLOP_PLAIN = 1264
# its adjoint (derivatives to order 7), counted the same way for the reduced
# formulas: r, 1/r and D_0..D_7: 23; the derivative recursion over the 85 (84)
# derivatives the contraction reads: 330; the reduced products: 25 x 16
# (24 x 16) -> source-role pass 1153, target-role pass 1121
FULL_ADJ_FLOP_REDUCED = 1153 + 1121
# the two-launch step of the full truncation: the forward that also keeps the
# target-side sums runs the source-role pass's pair loop (orders 0..4 from
# every moment, 1153), and so does the one-pass adjoint
FULL_SAVED_STEP_FLOP_REDUCED = 1153 + 1153


def full_truncation(plan, pairs, steps, Md, Xd, L, ot, torch, sched=None, wd=None, gM=None, gX=None):
    """Times the full-truncation forward on the benchmark plan: the given
    schedule, or the fastest of three over one launch each, then `steps`
    timed launches (HIP events on the launch stream); with weights and
    gradient arrays also its adjoint (both passes with the library's default
    schedule)."""
    stream = torch.cuda.current_stream()

    def timed(sched, n):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n):
            plan.multipole_batched_full(Md, Xd, L, sched=sched)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    default = ot.SCHED_W8P2 | ot.SCHED_PERSISTENT | ot.SCHED_LOCAL  # the library's AUTO for this truncation
    cands = {sc: sched_name(sc) for sc in (default, ot.SCHED_W8, ot.SCHED_W8P2)}
    if sched is not None:
        cands = {sched: sched_name(sched)}
    plan.multipole_batched_full(Md, Xd, L, sched=next(iter(cands)))  # warm-up
    best = min(cands, key=lambda sc: timed(sc, 1)) if len(cands) > 1 else next(iter(cands))
    ms = timed(best, steps)
    tf = pairs * FULL_FLOP_REDUCED / (ms * 1e-3) / 1e12
    log("full truncation %s: %.2f ms, %.3e pairs/s, %.2f TFLOP/s (reduced count)"
        % (cands[best], ms, pairs / (ms * 1e-3), tf))
    out = {"schedule": cands[best], "mean_ms": round(ms, 3), "pairs": pairs,
           "pairs_per_s": pairs / (ms * 1e-3),
           "flop_per_pair": FULL_FLOP_REDUCED, "flop_per_pair_plain": FULL_FLOP_PLAIN,
           "roofline": {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_TFLOPS, 4)}}
    if wd is not None and steps > 0:
        plan.multipole_backward_full(Md, Xd, wd, gM, gX)  # warm-up
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.multipole_backward_full(Md, Xd, wd, gM, gX)
        e1.record(stream)
        torch.cuda.synchronize()
        bms = e0.elapsed_time(e1) / steps
        btf = pairs * FULL_ADJ_FLOP_REDUCED / (bms * 1e-3) / 1e12
        log("full truncation adjoint: %.2f ms, %.2f TFLOP/s (reduced count); fwd+bwd %.3e pairs/s"
            % (bms, btf, pairs / ((ms + bms) * 1e-3)))
        out["adjoint"] = {"mean_ms": round(bms, 3), "flop_per_pair": FULL_ADJ_FLOP_REDUCED,
                          "roofline": {"bound": "alu", "achieved": round(btf, 3), "peak": PEAK_FP64_TFLOPS,
                                       "unit": "TFLOP/s", "frac": round(btf / PEAK_FP64_TFLOPS, 4)}}
        out["fwd_bwd_pairs_per_s"] = pairs / ((ms + bms) * 1e-3)
        # the two-launch step: forward with saved sums, one-pass adjoint
        Cs = torch.empty((ot.NSAVED, L.shape[1]), dtype=torch.float64, device=L.device)
        plan.multipole_batched_save(Md, Xd, L, Cs, full=True)  # warm-up
        plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX, full=True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.multipole_batched_save(Md, Xd, L, Cs, full=True)
            plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX, full=True)
        e1.record(stream)
        torch.cuda.synchronize()
        del Cs
        sms = e0.elapsed_time(e1) / steps
        stf = pairs * FULL_SAVED_STEP_FLOP_REDUCED / (sms * 1e-3) / 1e12
        log("full truncation two-launch step: %.2f ms (three launches %.2f), %.3e pairs/s, %.2f TFLOP/s"
            " (reduced count)" % (sms, ms + bms, pairs / (sms * 1e-3), stf))
        out["saved_step"] = {"mean_ms": round(sms, 3), "pairs_per_s": pairs / (sms * 1e-3),
                             "flop_per_pair": FULL_SAVED_STEP_FLOP_REDUCED,
                             "roofline": {"bound": "alu", "achieved": round(stf, 3), "peak": PEAK_FP64_TFLOPS,
                                          "unit": "TFLOP/s", "frac": round(stf / PEAK_FP64_TFLOPS, 4)}}
    return out


def two_level_step(n, steps, plan, batch, fs, Md, Xd, L, ot, synthetic, np, torch, dev, full=False):
    """A two-level step on the benchmark store, from the library's calls in
    sequence on one stream: upward pass to the (n/2)^3 parent level, fine
    interaction plus coarse substitutes for the missing neighbours, the
    parent level's interaction, downward pass into the fine coefficients,
    evaluation of force and energy. HIP events around the whole sequence.
    full=True: the three interaction passes with the full truncation (their
    default schedule)."""
    ch = synthetic.octree_children(n)
    Sp, S = ch.shape[0], n ** 3
    tree = ot.Tree(ch, S)
    parent = synthetic.parent_lattice(n, periodic=batch.get("period") is not None)
    pplan = ot.Plan.from_batch(parent)
    coarse, octant = synthetic.coarse_tables(n, batch)
    cpairs = plan.set_coarse(Sp, coarse, octant)
    f64 = dict(dtype=torch.float64, device=dev)
    Mp = torch.empty((20, Sp * 512), **f64)
    Xp = torch.empty((3, Sp * 512), **f64)
    Lp = torch.empty((20, Sp * 512), **f64)
    F = torch.empty((3, S * 512), **f64)
    W = torch.empty((S * 512,), **f64)

    def step():
        tree.m2m(Md, Xd, Mp, Xp)
        if full:
            plan.multipole_batched_full(Md, Xd, L)
        else:
            plan.multipole_batched(Md, Xd, L, sched=fs)
        plan.coarse_fine(Xd, Mp, Xp, L, full=full)
        if full:
            pplan.multipole_batched_full(Mp, Xp, Lp)
        else:
            pplan.multipole_batched(Mp, Xp, Lp)
        tree.l2l(Lp, Xp, Xd, L)
        ot.ot_fmm_evaluate(Md, L, F, W)

    step()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    fine_pairs, parent_pairs = plan.pairs(), pplan.pairs()
    total = fine_pairs + cpairs + parent_pairs
    log("two-level step%s %.2f ms: %d fine + %d coarse + %d parent-level pairs" % (
        " (full truncation)" if full else "", ms, fine_pairs, cpairs, parent_pairs))
    tree.close()
    pplan.close()
    return {"mean_ms": round(ms, 3), "fine_pairs": fine_pairs, "coarse_pairs": cpairs,
            "parent_pairs": parent_pairs, "pairs_per_s": total / (ms * 1e-3),
            "passes": ["m2m", "forward (fine)", "coarse_fine", "forward (parent level)", "l2l",
                       "evaluate"]}


def per_subgrid_comparison(n, ot, synthetic, np, torch, dev):
    """Forward on n^3 sub-grids (15% missing 1..9 neighbours): one batched
    launch vs one single-block launch per target on pre-gathered 24^3 halos
    (gather not timed), on 1, 8 and 32 streams used round-robin."""
    batch, M, X = synthetic.config3(n)
    plan = ot.Plan.from_batch(batch)
    pairs = plan.pairs()
    T = batch["T"]
    Md = torch.from_numpy(M).to(dev)
    Xd = torch.from_numpy(X).to(dev)
    L = torch.empty((20, T * 512), dtype=torch.float64, device=dev)
    f, _ = plan.autotune(Md, Xd, L)
    times = []
    for _ in range(3):
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record()
        plan.multipole_batched(Md, Xd, L, sched=f)
        s1.record()
        torch.cuda.synchronize()
        times.append(s0.elapsed_time(s1))
    batched_ms = sorted(times)[1]
    log("per-sub-grid comparison: batched forward %.2f ms" % batched_ms)

    # gather every target's halo: missing neighbours -> zero moments, centres
    # kept finite; periodic images shifted
    loc = np.arange(512)
    lx, ly, lz = loc % 8, (loc // 8) % 8, loc // 64
    hidx = np.empty((27, 512), np.int64)
    for slot in range(27):
        sx, sy, sz = slot % 3, (slot // 3) % 3, slot // 9
        hidx[slot] = (8 * sx + lx) + 24 * (8 * sy + ly) + 576 * (8 * sz + lz)
    nbr = batch["nbr"]
    src = np.where(nbr >= 0, nbr, nbr[:, 13:14])
    gidx = (src[:, :, None] * 512 + loc[None, None, :]).reshape(T, 27 * 512)
    order = np.argsort(hidx.reshape(-1))
    gidx = torch.from_numpy(gidx[:, order]).to(dev)             # (T, 13824) store index
    miss = torch.from_numpy((nbr < 0)[:, :, None].repeat(512, 2).reshape(T, -1)[:, order]).to(dev)
    shift = torch.from_numpy(
        (batch["shift"].astype(np.float64) * batch["period"][None, None, :]).repeat(512, 1)
        .reshape(T, 27, 512, 3).reshape(T, 27 * 512, 3)[:, order]).to(dev)   # (T, 13824, 3)
    Mh = torch.empty((T, 20, 13824), dtype=torch.float64, device=dev)
    Xh = torch.empty((T, 3, 13824), dtype=torch.float64, device=dev)
    for t0 in range(0, T, 256):
        t1 = min(T, t0 + 256)
        g = gidx[t0:t1]
        mm = Md[:, g].permute(1, 0, 2)
        mm = torch.where(miss[t0:t1, None, :], torch.zeros_like(mm), mm)
        Mh[t0:t1] = mm
        xx = Xd[:, g].permute(1, 0, 2) + shift[t0:t1].permute(0, 2, 1)
        xx = torch.where(miss[t0:t1, None, :], xx + 1.0e6, xx)
        Xh[t0:t1] = xx
    Lh = torch.empty((T, 20, 512), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    res = {"workload": "batched multipole forward, %d^3 sub-grids, 15%% missing 1-9 neighbours"
                       % n, "targets": T, "pairs": pairs,
           "batched_ms": round(batched_ms, 3),
           "batched_pairs_per_s": pairs / (batched_ms * 1e-3)}
    for nstreams in (1, 8, 32):
        streams = [torch.cuda.Stream() for _ in range(nstreams)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(T):
            ot.ot_fmm_multipole(Mh[t], Xh[t], Lh[t], stream=streams[t % nstreams])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        res["per_subgrid_%dstream_ms" % nstreams] = round(ms, 2)
        res["speedup_vs_%dstream" % nstreams] = round(ms / batched_ms, 2)
        log("per-sub-grid launches on %2d stream(s): %.1f ms (%.1fx slower)"
            % (nstreams, ms, ms / batched_ms))
    # the same launches captured into one graph (fork / join over the
    # streams, round-robin), replayed: the per-launch cost without host
    # dispatch through Python and the runtime
    Lg = torch.empty_like(Lh)
    for nstreams in (1, 8, 32):
        cap = torch.cuda.Stream()
        side = [torch.cuda.Stream() for _ in range(nstreams - 1)]
        graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=cap):
            cur = torch.cuda.current_stream()
            lanes = [cur] + side
            for sd in side:
                sd.wait_stream(cur)
            for t in range(T):
                ot.ot_fmm_multipole(Mh[t], Xh[t], Lg[t], stream=lanes[t % nstreams])
            for sd in side:
                cur.wait_stream(sd)
        times = []
        for _ in range(3):
            Lg.fill_(float("nan"))
            g0 = torch.cuda.Event(enable_timing=True)
            g1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            g0.record()
            graph.replay()
            g1.record()
            torch.cuda.synchronize()
            times.append(g0.elapsed_time(g1))
        ms = sorted(times)[1]
        res["per_subgrid_graph_%dstream_ms" % nstreams] = round(ms, 2)
        res["speedup_vs_graph_%dstream" % nstreams] = round(ms / batched_ms, 2)
        res["graph_%dstream_bitwise_equal_to_stream_launches" % nstreams] = bool(torch.equal(Lg, Lh))
        log("per-sub-grid launches in one graph on %2d stream(s): %.1f ms (%.1fx slower)"
            % (nstreams, ms, ms / batched_ms))
        del graph
    del Lg
    # the same launches as futures completed by event polling (32 pool
    # streams, 4 worker threads polling between tasks), waited for by polling
    Lf = torch.empty_like(Lh)
    ex = ot.Executor(nstreams=32, nworkers=4)
    for s in range(32):
        ex.stream(s)  # create the pool streams outside the timed region
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    futs = [ex.multipole_async(Mh[t], Xh[t], Lf[t]) for t in range(T)]
    for f in futs:
        f.wait(120.0)
    ms = (time.perf_counter() - t0) * 1e3
    del futs
    ex.close()
    res["per_subgrid_futures_32stream_ms"] = round(ms, 2)
    res["speedup_vs_futures_32stream"] = round(ms / batched_ms, 2)
    res["futures_bitwise_equal_to_stream_launches"] = bool(torch.equal(Lf, Lh))
    log("per-sub-grid launches as polled futures (32 streams): %.1f ms (%.1fx slower)"
        % (ms, ms / batched_ms))
    del Lf
    # same numbers as the batched launch up to summation order (the missing
    # cells add exact zeros): per target and output order, max |diff| / max |L|
    Lb = L.reshape(20, T, 512).permute(1, 0, 2)
    worst = 0.0
    for g in ([0], [1, 2, 3], list(range(4, 10)), list(range(10, 20))):
        d = (Lh[:, g] - Lb[:, g]).abs().amax(dim=(1, 2))
        sc = Lb[:, g].abs().amax(dim=(1, 2))
        worst = max(worst, float((d / sc).max()))
    res["max_rel_diff_vs_batched"] = worst
    del Mh, Xh, Lh
    torch.cuda.empty_cache()
    return res


def cpu_baseline(batch, M, X, w, seconds, np):
    """The CPU oracle (plain C, OpenMP over all host cores) on a bounded
    sample of the benchmark workload: forward of k target sub-grids plus the
    adjoint of the same k store sub-grids, k doubled until the budget is
    reached. Value: sampled forward pairs / (forward + adjoint time)."""
    import oracle
    from oracle import max_threads
    rng = np.random.default_rng(123)
    order = rng.permutation(batch["T"])
    nbr = batch["nbr"]
    slot_pairs = _slot_pairs(np)
    k, spent, pairs, used = 1, 0.0, 0, 0
    while True:
        sel = order[used:used + k].astype(np.int32)
        t0 = time.perf_counter()
        oracle.batched_forward(batch, M, X, tsel=sel)
        oracle.batched_backward(batch, M, X, w, ssel=sel)
        spent += time.perf_counter() - t0
        pairs += int(sum(slot_pairs[s] for t in sel for s in range(27) if nbr[t, s] >= 0))
        used += k
        if spent >= seconds or used + 2 * k > batch["T"]:
            break
        k = 2 * k if spent < seconds / 4 else k
    log("cpu oracle: %d sub-grids, %.1f s, %d threads" % (used, spent, max_threads()))
    # one thread on the first sampled sub-grid: the per-core rate
    sel = order[:1].astype(np.int32)
    t0 = time.perf_counter()
    oracle.batched_forward(batch, M, X, tsel=sel, nthreads=1)
    oracle.batched_backward(batch, M, X, w, ssel=sel, nthreads=1)
    one = time.perf_counter() - t0
    one_pairs = int(sum(slot_pairs[s] for s in range(27) if nbr[sel[0], s] >= 0))
    log("cpu oracle, one thread: %.1f s" % one)
    # the single-block workloads, timed in full: monopole and multipole
    # interaction of one 24^3 halo block (921,088 pairs each)
    import synthetic
    blocks = {}
    for name, b, mom in (("monopole_block", synthetic.monopole_block(1001), "mass"),
                         ("multipole_block", synthetic.multipole_block(1002), "M")):
        m = b[mom] if mom == "M" else b[mom][None]
        t0 = time.perf_counter()
        oracle.block_forward(m, b["com"])
        dt = time.perf_counter() - t0
        blocks[name] = {"pairs": 921088, "s": round(dt, 4), "pairs_per_s": 921088 / dt}
        log("cpu oracle, %s: %.3f s" % (name, dt))
    total = sum(slot_pairs[s] for t in range(batch["T"]) for s in range(27) if nbr[t, s] >= 0)
    return {"value": pairs / spent, "unit": "cell-pair interactions/s", "cores": max_threads(),
            "kind": "oracle",
            "sample": "fwd of %d sampled target sub-grids + adjoint of the same %d store "
                      "sub-grids of the benchmark workload (%d pairs, %.1f s); its rate, extrapolated "
                      "by the exact pair count, gives %.0f s for one forward+adjoint step of all %d pairs"
                      % (used, used, pairs, spent, total * spent / pairs, total),
            "extrapolated_step_s": round(total * spent / pairs, 1),
            "one_core_value": one_pairs / one,
            "single_block_forward": blocks,
            "cpu_model": _cpu_model(),
            "host_cpus": len(os.sched_getaffinity(0))}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _slot_pairs(np):
    c = np.arange(512)
    loc = np.stack([c % 8, (c // 8) % 8, c // 64], axis=1)
    ti = loc + 8
    out = []
    for slot in range(27):
        off = 8 * np.array([slot % 3, (slot // 3) % 3, slot // 9])
        tj = loc + off
        dd = tj[None, :, :] - ti[:, None, :]
        p = tj[None, :, :] // 2 - ti[:, None, :] // 2
        out.append(int(np.count_nonzero(((dd * dd).sum(-1) > 16) & ((p * p).sum(-1) <= 16))))
    return out


if __name__ == "__main__":
    main()
