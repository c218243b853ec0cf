"""Benchmark: cell-updates/s of the AMR advance + ghost fill on one MI355X.

Workload (default): uniform level 5 of the unit square, 1024 patches of
32x32 cells with 2 ghost layers, FP64 scalar advection in the swirling
deformational field, seeded sum of 8 Gaussians, 500 steps.  A "step" is
one coarse step of the whole path: ghost fill + advance of every patch.

The headline uses the fused form: one advance kernel per level-step that
gathers its ghost values on the fly from neighbour interiors (no fill
launch), chunks of 50 coarse steps captured once and replayed from a
hipGraph.  The plain per-level launch form (a fill launch and an advance
launch per level-step), the same fused kernels launched from the host, and
the persistent single-kernel form are timed on the same workload and
reported beside it.

Output: one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/sec (advance+ghost fill) at 1 GPU; % HBM roofline; fused vs per-level"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1703_03116_amd/csrc/fc_kernels.hip", "paper_1703_03116_amd/csrc/fc_internal.h"]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(npatch, mx, F):
    """Read every patch tile with its halo once, write its interior once."""
    N = mx + 4
    return npatch * F * 8 * (N * N + mx * mx)


def traffic_from_profiles(nt):
    """HBM bytes per launch of the level-step kernel from the committed
    counter summary, if it was taken on the current kernel source and launch
    variant."""
    p = os.path.join(ROOT, "profiles", "traffic_level_step_swirl_l5.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_sha") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch", {}).get(str(nt))


def stream_copy_gbs(nbytes=1 << 30, reps=5):
    """Plain device-to-device copy rate on this GPU (read + write bytes per
    second), buffers far larger than the 256 MB Infinity Cache."""
    import torch
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 8 * reps / sec / 1e9


def cpu_baseline(w, budget_s=15.0):
    """The oracle, as is, on a bounded sample of the same workload."""
    from oracle import oracle as O
    nth = min(os.cpu_count() or 1, 16)
    O.set_threads(nth)
    o = O.from_workload(w)
    dt = w["dt_coarse"]
    cells = len(w["leaves"]) * w["mx"] ** 2
    t0 = time.perf_counter()
    o.coarse_step(0.0, dt)
    one = time.perf_counter() - t0
    n = max(1, min(w["steps"] - 1, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    for s in range(n):
        o.coarse_step((s + 1) * dt, dt)
    el = time.perf_counter() - t0
    return {"value": cells * n / el, "unit": "cell-updates/s", "cores": O.max_threads(), "kind": "oracle",
            "sample": f"{n} steps of the same {len(w['leaves'])}-patch workload (after 1 untimed step)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=500,
                    help="untimed steps first (the GPU's clocks settle over the first few milliseconds of load)")
    ap.add_argument("--level", type=int, default=5)
    ap.add_argument("--mx", type=int, default=32)
    ap.add_argument("--workload", default="swirl_uniform",
                    choices=["swirl_uniform", "swirl_amr", "dam_break", "adjoint"],
                    help="swirl_uniform (default; --level sets its size), swirl_amr (levels 3-7, regrid "
                         "every 2 coarse steps), dam_break (shallow water, levels 2-6, 16x16), adjoint "
                         "(gradient of an L2 misfit, uniform level 6, 256 steps, checkpoints every 16)")
    ap.add_argument("--threads", type=int, default=0,
                    help="threads per patch of the advance kernels (0: autotune)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-level", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU exchange is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1703_03116_amd import binding as B
    from workloads import synth as S

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy kernel of known size: reads 256 MiB, writes 256 MiB
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "adjoint":
        return adjoint_workload(args)
    if args.workload != "swirl_uniform":
        return other_workload(args)
    w = S.workload("swirl_uniform", level=args.level, mx=args.mx, steps=args.steps)
    P, mx, F = len(w["leaves"]), w["mx"], 1
    dt = w["dt_coarse"]
    cells_per_step = P * mx * mx
    ps = B.from_workload(w)
    if args.threads:
        ps.set_variant(args.threads)
        nt = args.threads
    else:
        nt = ps.autotune()
    stream = torch.cuda.current_stream()

    def timed(store, mode, k):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        store.coarse_steps(dt, k, mode)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    # headline: one ghost-gathering advance kernel per level-step, chunks of
    # coarse steps replayed from a captured hipGraph; the graphs the timed
    # steps replay are captured (one-time set-up, timed apart) after the
    # warm-up steps and before the timed region
    ps.coarse_steps(dt, args.warmup, "graph")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ps.prepare_steps(dt, args.steps, "graph")
    torch.cuda.synchronize()
    capture_ms = 1e3 * (time.perf_counter() - t0)
    sec = timed(ps, "graph", args.steps)
    ps.check()
    value = cells_per_step * args.steps / sec
    # uniform level: one level-step kernel launch per coarse step (plus one
    # small bookkeeping node per 50 steps); the average launch duration over
    # the timed region, measured with events on the stream the graph runs on
    # (node gaps included)
    avg_launch = sec / args.steps
    bpl = algorithmic_bytes(P, mx, F)
    achieved = bpl / avg_launch / 1e9
    traffic = traffic_from_profiles(nt)

    forms = {}
    if not args.no_per_level:
        for mode in ("per_level", "persistent_graph", "fused_levels"):
            ps2 = B.from_workload(w)
            ps2.set_variant(nt)
            ps2.coarse_steps(dt, args.warmup, mode)
            ps2.prepare_steps(dt, args.steps, mode)
            s2 = timed(ps2, mode, args.steps)
            ps2.check()
            forms[mode] = {"value": cells_per_step * args.steps / s2, "ms_per_step": 1e3 * s2 / args.steps}
            del ps2
    per_level = forms.get("per_level")

    copy_gbs = stream_copy_gbs()
    cpu = None if args.no_cpu_baseline else cpu_baseline(w)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"swirl_uniform_l{args.level}: {P} patches of {mx}x{mx} cells, 2 ghost layers, "
                               f"FP64 scalar advection, swirl field T=1, seeded 8-Gaussian data, "
                               f"{args.steps} steps",
                   "patches": P, "mx": mx, "cells": cells_per_step,
                   "mode": "fused: one ghost-gathering advance kernel per level-step, replayed from a hipGraph",
                   "threads_per_patch": nt, "graph_capture_ms": capture_ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "level_step_kernel<32,%d,0>" % nt, "bytes_per_launch": bpl,
                     "avg_launch_ms": 1e3 * avg_launch,
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "per_level": per_level,
        "other_forms": forms,
        "fused_over_per_level": (value / per_level["value"]) if per_level else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def other_workload(args):
    """Adaptive workloads: cell updates over advance + fill time (regrid timed
    apart), fused graph form and per-level form, one JSON line."""
    import numpy as np
    import torch
    from paper_1703_03116_amd import binding as B
    from paper_1703_03116_amd.amr import run_adaptive
    from workloads import synth as S

    res = {}
    for mode in ("graph", "per_level"):
        if args.workload == "swirl_amr":
            w = S.workload("swirl_amr")
            ps = B.from_workload(w, capacity=4 ** w["lmax"])
            nt = ps.autotune()
            tm = {}
            run_adaptive(ps, w["dt_coarse"], 2, regrid_every=2, mode=mode)  # warm-up
            cells = run_adaptive(ps, w["dt_coarse"], args.steps, regrid_every=2, mode=mode, timings=tm)
            res[mode] = {"value": cells / tm["advance"], "advance_s": tm["advance"],
                         "regrid_s": tm.get("regrid", 0.0), "patches_end": ps.nleaves}
        else:
            w = S.workload("dam_break")
            ps = B.from_workload(w)
            nt = ps.autotune()
            lv = np.asarray(w["leaves"])[:, 0]
            dt = 0.6 / (w["mx"] << w["lmin"]) / 2.5   # finest-level Courant number <= 0.6 for speeds <= 2.5
            per_step = sum(int((lv == l).sum()) * w["mx"] ** 2 * (1 << (l - w["lmin"])) for l in np.unique(lv))
            ps.coarse_steps(dt, 2, mode)
            torch.cuda.synchronize()
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ps.coarse_steps(dt, args.steps, mode)
            e1.record(stream)
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) / 1e3
            ps.check()
            res[mode] = {"value": per_step * args.steps / sec, "ms_per_coarse_step": 1e3 * sec / args.steps,
                         "patches": len(lv)}
    out = {"metric": METRIC, "value": res["graph"]["value"], "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 2, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic", "config": {"workload": args.workload, "threads_per_patch": nt},
           "fused_graph": res["graph"], "per_level": res["per_level"],
           "fused_over_per_level": res["graph"]["value"] / res["per_level"]["value"]}
    print(json.dumps(out), flush=True)


def adjoint_workload(args):
    """Gradient of L = 1/2 ||q(T) - q_target||^2 with respect to q0: forward
    pass with checkpoints, then per segment recomputation and the hand-written
    adjoint steps.  Value: forward-equivalent cell updates per second of
    gradient time (cells x steps / seconds); the forward pass alone and the
    adjoint step kernel's share are reported beside it."""
    import torch
    from paper_1703_03116_amd import binding as B
    from paper_1703_03116_amd.adjoint import loss_and_grad
    from workloads import synth as S

    level, mx, n, every = 6, 32, (args.steps if args.steps != 500 else 256), 16
    L = S.uniform_leaves(level)
    q0 = torch.tensor(S.sample_on_leaves(S.gaussians(S.gaussian_params(5)), L, mx), device="cuda")
    qt = torch.tensor(S.sample_on_leaves(S.gaussians(S.gaussian_params(6)), L, mx), device="cuda")
    dt = 0.9 / (mx << level)
    ps = B.PatchStore(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter="mc")
    nt = ps.autotune()
    loss_and_grad(ps, q0, qt, level, dt, 16, every)  # warm-up (graphs, kernels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Lv, g = loss_and_grad(ps, q0, qt, level, dt, n, every)
    torch.cuda.synchronize()
    grad_s = time.perf_counter() - t0
    # the same gradient with every state kept in HBM (n solution copies,
    # 8.6 GB at level 6 and 256 steps): no recomputation
    loss_and_grad(ps, q0, qt, level, dt, n, 1)  # warm-up at full length: the n state buffers come from the
    torch.cuda.synchronize()                    # caching allocator afterwards, not from fresh allocations
    t0 = time.perf_counter()
    _, g1 = loss_and_grad(ps, q0, qt, level, dt, n, 1)
    torch.cuda.synchronize()
    grad1_s = time.perf_counter() - t0
    same = bool(torch.equal(g, g1))
    del g1
    torch.cuda.empty_cache()
    ps.time = 0.0
    ps.set_interior(q0)
    ps.prepare_steps(dt, n, "graph")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ps.coarse_steps(dt, n, "graph")
    torch.cuda.synchronize()
    fwd_s = time.perf_counter() - t0
    ps.check()
    cells = len(L) * mx * mx
    out = {"metric": "cell-updates/sec of the gradient (forward + recompute + adjoint) at 1 GPU",
           "value": cells * n / grad_s, "unit": "cell-updates/s", "n_gpus": 1, "steps": n, "warmup": 1,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"adjoint: uniform level {level}, {len(L)} patches of {mx}x{mx}, swirl, MC limiter, "
                                  f"{n} steps, checkpoint every {every}", "threads_per_patch": nt},
           "gradient_s": grad_s, "forward_s": fwd_s, "gradient_over_forward": grad_s / fwd_s,
           "all_states_resident": {"gradient_s": grad1_s, "gradient_over_forward": grad1_s / fwd_s,
                                   "bitwise_equal_gradient": same},
           "loss": float(Lv), "grad_norm": float(g.norm())}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
