"""Benchmark: cell-updates/s of the AMR advance + ghost fill on one MI355X.

Default workload: adaptive levels 3-7 of the unit square with 32x32 patches
and 2 ghost layers, FP64 scalar advection in the swirling deformational
field, seeded sum of 8 Gaussians, multirate subcycling (31 level-steps per
coarse step), regrid every 2 coarse steps by tagging |grad q| > 0.05.  A
"step" is one coarse step: ghost fill + advance of every patch on every
level.  The metric counts cell updates (sum over level-steps of patches x
mx^2) over the advance + fill time, measured with HIP events on the stream
the work runs on; regridding (tag, host adaptation, transfer, and the graph
capture a new mesh needs) is timed apart, as the paper reports it.

The headline uses the fused form: one advance kernel per level-step that
gathers its ghost values on the fly from neighbour interiors (no fill
launch), the coarse steps between two regrids captured as one hipGraph and
replayed.  The plain per-level form (a fill launch and an advance launch per
level-step) is timed on the same meshes.  The line also carries the HBM
roofline of the same kernel on uniform level 8 (65536 patches, 1.36 GB per
buffer, far beyond the 256 MB Infinity Cache) and the CPU oracle's rate.

Other workloads: --workload swirl_uniform (--level sets the size),
dam_break, adjoint.  Output: one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
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


def level_step_name(mx, nt, seg):
    """The scalar level-step kernel as instantiated (last argument: cells per
    sweep segment, 0 for the default length)."""
    default = max(4, min(mx, 2 * mx * mx // nt))
    return "level_step_kernel<%d,%d,0,%d>" % (mx, nt, 0 if seg == default else seg)


def algorithmic_bytes(npatch, mx, F):
    """Read every patch tile with its halo once, write its interior once."""
    N = mx + 4
    return npatch * F * 8 * (N * N + mx * mx)


def traffic_from_profiles(name, nt):
    """Measured HBM bytes per algorithmic byte of the level-step kernel from a
    committed counter summary, if it was taken on the current kernel source
    and launch variant (else None)."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_sha") != kernel_hash():
        return None
    return d.get("hbm_over_algorithmic", {}).get(str(nt))


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


def host_cpu():
    """nproc, the CPU model and the cores this process may use (at most 16:
    the host share of one GPU)."""
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
    except Exception:
        nproc = os.cpu_count() or 1
    usable = min(len(os.sched_getaffinity(0)), 16)
    return nproc, model, usable


def cpu_baseline(w, budget_s=12.0):
    """The oracle, as is, on a bounded sample of the same workload: every
    usable core (OpenMP over patches) on whole coarse steps of the initial
    mesh, and one core on one level-step (fill + advance) of the most
    populated level."""
    import numpy as np
    from oracle import oracle as O
    nproc, model, usable = host_cpu()
    O.set_threads(usable)
    o = O.from_workload(w)
    dt = w["dt_coarse"]
    lv = np.asarray(w["leaves"])[:, 0]
    lmin = w["lmin"]
    per_step = sum(int((lv == l).sum()) * w["mx"] ** 2 * (1 << (int(l) - lmin)) for l in np.unique(lv))
    t0 = time.perf_counter()
    o.coarse_step(0.0, dt)
    one = time.perf_counter() - t0
    n = max(1, min(w["steps"] - 1, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    for s in range(n):
        o.coarse_step((s + 1) * dt, dt)
    el = time.perf_counter() - t0
    allc = per_step * n / el
    threads = O.max_threads()
    # one core: fill + advance of the most populated level once
    O.set_threads(1)
    lbig = int(np.bincount(lv).argmax())
    o2 = O.from_workload(w)
    dtl = dt / (1 << (lbig - lmin))
    t0 = time.perf_counter()
    o2.ghost_fill(lbig, lbig, 1.0)
    o2.advance_level(lbig, 0.0, dtl)
    el1 = time.perf_counter() - t0
    one_core = int((lv == lbig).sum()) * w["mx"] ** 2 / el1
    return {"value": allc, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} coarse steps of the initial {len(lv)}-patch mesh (after 1 untimed step), "
                      f"{threads} threads",
            "nproc": nproc, "cpu_model": model,
            "one_core": {"value": one_core, "unit": "cell-updates/s",
                         "sample": f"one level-step (fill + advance) of level {lbig}, "
                                   f"{int((lv == lbig).sum())} patches, 1 thread"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed coarse steps (default: 40 for swirl_amr, 500 for swirl_uniform, 100 for dam_break)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed coarse steps first (default: 4 for swirl_amr, 500 for swirl_uniform)")
    ap.add_argument("--level", type=int, default=5, help="level of --workload swirl_uniform")
    ap.add_argument("--mx", type=int, default=32)
    ap.add_argument("--workload", default="swirl_amr",
                    choices=["swirl_amr", "swirl_uniform", "dam_break", "adjoint", "mapped_uniform"],
                    help="swirl_amr (default: levels 3-7, regrid every 2 coarse steps), swirl_uniform (--level "
                         "sets its size), dam_break (shallow water, levels 2-6, 16x16), adjoint (gradient of an "
                         "L2 misfit, uniform level 6, 256 steps, checkpoints every 16), mapped_uniform (the swirl "
                         "on a mapped grid, --level, --map-alpha; fill and capacity-form advance timed apart)")
    ap.add_argument("--map-alpha", type=float, default=0.1, help="mapping amplitude of --workload mapped_uniform")
    ap.add_argument("--tile", type=int, default=0,
                    help="cells per sweep segment of the scalar advance with --threads (0: the default)")
    ap.add_argument("--threads", type=int, default=0,
                    help="threads per patch of the advance kernels (0: autotune)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-level", action="store_true")
    ap.add_argument("--no-l8", action="store_true", help="skip the uniform level-8 HBM-roofline field")
    ap.add_argument("--l8-steps", type=int, default=40)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run three plain 256 MiB device copies (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on one GPU; its multi-GPU exchange is designed, not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
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
    if args.workload == "dam_break":
        return dam_break_workload(args)
    if args.workload == "mapped_uniform":
        return mapped_workload(args)
    if args.workload == "swirl_uniform":
        steps = args.steps if args.steps is not None else 500
        warm = args.warmup if args.warmup is not None else 500
        out = uniform_workload(args.level, args.mx, steps, warm, args.threads, not args.no_per_level, args.tile)
        if not args.no_cpu_baseline:
            from workloads import synth as S
            w = S.workload("swirl_uniform", level=args.level, mx=args.mx, steps=steps)
            out["cpu_baseline"] = cpu_baseline(w)
        print(json.dumps(out), flush=True)
        return
    return amr_workload(args)


def uniform_workload(level, mx, steps, warmup, threads=0, forms=True, tile=0):
    """Uniform level of the swirl workload, graph form (one level-step kernel
    per coarse step, 50-step chunks plus one graph for the rest replayed);
    returns the fields of a bench line (no cpu_baseline)."""
    import torch
    from paper_1703_03116_amd import binding as B
    from workloads import synth as S

    w = S.workload("swirl_uniform", level=level, mx=mx, steps=steps)
    P, F = len(w["leaves"]), 1
    dt = w["dt_coarse"]
    cells_per_step = P * mx * mx
    ps = B.from_workload(w)
    if threads:
        ps.set_variant(threads)
        ps.set_tile(tile)
    else:
        ps.autotune()
    nt, seg = ps.launch()
    stream = torch.cuda.current_stream()

    def timed(store, mode, k):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        store.coarse_steps(dt, k, mode)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    # the graphs the timed steps replay are captured (one-time set-up, timed
    # apart) after the warm-up steps and before the timed region
    ps.coarse_steps(dt, warmup, "graph")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ps.prepare_steps(dt, steps, "graph")
    torch.cuda.synchronize()
    capture_ms = 1e3 * (time.perf_counter() - t0)
    sec = timed(ps, "graph", steps)
    ps.check()
    value = cells_per_step * steps / sec
    # one level-step kernel launch per coarse step (plus one bookkeeping node
    # per replayed graph): the average launch duration over the timed region,
    # measured with events on the stream the graph runs on (node gaps included)
    avg_launch = sec / steps
    bpl = algorithmic_bytes(P, mx, F)
    achieved = bpl / avg_launch / 1e9
    ratio = traffic_from_profiles(f"traffic_level_step_swirl_l{level}.json", nt)
    del ps
    forms_out = {}
    if forms:
        for mode in ("per_level", "fused_levels"):
            ps2 = B.from_workload(w)
            ps2.set_variant(nt)
            ps2.set_tile(seg)
            ps2.coarse_steps(dt, min(warmup, 50), mode)
            ps2.prepare_steps(dt, steps, mode)
            s2 = timed(ps2, mode, steps)
            ps2.check()
            forms_out[mode] = {"value": cells_per_step * steps / s2, "ms_per_step": 1e3 * s2 / steps}
            del ps2
    torch.cuda.empty_cache()
    copy_gbs = stream_copy_gbs()
    per_level = forms_out.get("per_level")
    return {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": 1e3 * sec / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"swirl_uniform_l{level}: {P} patches of {mx}x{mx} cells, 2 ghost layers, "
                               f"FP64 scalar advection, swirl field T=1, seeded 8-Gaussian data, {steps} steps",
                   "patches": P, "mx": mx, "cells": cells_per_step,
                   "mode": "fused: one ghost-gathering advance kernel per level-step, replayed from a hipGraph",
                   "threads_per_patch": nt, "sweep_segment_cells": seg, "graph_capture_ms": capture_ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": (ratio * bpl) if ratio else None,
                     "kernel": level_step_name(mx, nt, seg), "bytes_per_launch": bpl,
                     "avg_launch_ms": 1e3 * avg_launch, "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "per_level": per_level,
        "other_forms": forms_out,
        "fused_over_per_level": (value / per_level["value"]) if per_level else None,
    }


def mapped_workload(args):
    """Uniform level of the swirl workload on the mapped grid X = (xi, eta) +
    alpha sin(2 pi xi) sin(2 pi eta) (1, 1), per-level form: per step a fill
    launch and a capacity-form advance launch, each bracketed by HIP events
    on the stream it runs on.  The roofline is the advance kernel's
    (algorithmic bytes: the tile with its halo read once, the interior
    written once; the per-level capacity table is a few KB); its HBM traffic
    comes from the committed counter summary while the kernel source is the
    one it was taken on."""
    import math
    import torch
    from paper_1703_03116_amd import binding as B
    from workloads import synth as S

    level, mx, alpha = args.level, args.mx, args.map_alpha
    steps = args.steps if args.steps is not None else 40
    warm = args.warmup if args.warmup is not None else 10
    w = S.workload("swirl_uniform", level=level, mx=mx, steps=steps)
    P = len(w["leaves"])
    # the smallest cells (area factor down to 1 - 2 pi |alpha|) bound the step
    dt = w["dt_coarse"] * (1.0 - 2.0 * math.pi * abs(alpha))
    ps = B.PatchStore(w["leaves"], mx=mx, velocity="swirl", vel_params=w["vel_params"], min_level=level,
                      max_level=level, map_alpha=alpha)
    ps.set_interior(w["q0"])
    if args.threads:
        ps.set_variant(args.threads)
        nt = args.threads
    else:
        nt = ps.autotune()
    stream = torch.cuda.current_stream()
    cfl = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = 0.0
    for _ in range(warm):
        ps.ghost_fill()
        ps.advance_level(level, t, dt, cfl)
        t += dt
    torch.cuda.synchronize()
    # timed steps without the Courant reduction, so that each event pair
    # brackets one kernel (the warm-up steps above recorded the Courant number)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record(stream)
        ps.ghost_fill()
        ev[k][1].record(stream)
        ps.advance_level(level, t, dt)
        ev[k][2].record(stream)
        t += dt
    torch.cuda.synchronize()
    ps.check()
    fill_s = sum(e[0].elapsed_time(e[1]) for e in ev) / 1e3
    adv_s = sum(e[1].elapsed_time(e[2]) for e in ev) / 1e3
    sec = ev[0][0].elapsed_time(ev[-1][2]) / 1e3
    cells = P * mx * mx
    bpl = algorithmic_bytes(P, mx, 1)
    achieved = bpl / (adv_s / steps) / 1e9
    ratio = traffic_from_profiles(f"traffic_advance_mapped_l{level}.json", nt)
    copy_gbs = stream_copy_gbs()
    out = {
        "metric": METRIC, "value": cells * steps / sec, "unit": "cell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warm, "ms_per_step": 1e3 * sec / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"mapped_uniform_l{level}: {P} patches of {mx}x{mx} cells on the mapped grid "
                               f"alpha={alpha}, 2 ghost layers, FP64 scalar advection in capacity form, swirl "
                               f"field T=1, seeded 8-Gaussian data, {steps} steps",
                   "patches": P, "mx": mx, "cells": cells, "map_alpha": alpha,
                   "mode": "per_level: a fill launch and a capacity-form advance launch per step",
                   "threads_per_patch": nt, "max_courant": float(cfl.item())},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": (ratio * bpl) if ratio else None,
                     "kernel": "advance_mapped_kernel<%d,%d,false>" % (mx, nt), "bytes_per_launch": bpl,
                     "avg_launch_ms": 1e3 * adv_s / steps, "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "fill": {"avg_launch_ms": 1e3 * fill_s / steps},
    }
    print(json.dumps(out), flush=True)


def amr_workload(args):
    """The default line: adaptive swirl, levels 3-7 (see the module
    docstring), graph form against the per-level form on the same meshes."""
    import torch
    from paper_1703_03116_amd import binding as B
    from paper_1703_03116_amd.amr import run_adaptive
    from workloads import synth as S

    steps = args.steps if args.steps is not None else 40
    warm = args.warmup if args.warmup is not None else 4
    w = S.workload("swirl_amr", steps=steps)
    dt = w["dt_coarse"]
    cap = 4 ** w["lmax"]
    ps = B.from_workload(w, capacity=cap)
    if args.threads:
        nt, seg = args.threads, args.tile
    else:
        ps.autotune()
        nt, seg = ps.launch()
    del ps
    res = {}
    for mode in ("graph",) + (() if args.no_per_level else ("per_level",)):
        ps = B.from_workload(w, capacity=cap)
        ps.set_variant(nt)
        ps.set_tile(seg)
        run_adaptive(ps, dt, warm, regrid_every=2, mode=mode)
        tm = {}
        cells = run_adaptive(ps, dt, steps, regrid_every=2, mode=mode, timings=tm)
        ps.check()
        res[mode] = {"value": cells / tm["advance"], "ms_per_step": 1e3 * tm["advance"] / steps,
                     "advance_s": tm["advance"], "regrid_s": tm["regrid"], "regrids": tm["regrids"],
                     "launches": tm["launches"], "bytes": tm["bytes"], "cells": cells,
                     "patches_end": ps.nleaves}
        del ps
        torch.cuda.empty_cache()
    g = res["graph"]
    achieved = g["bytes"] / g["advance_s"] / 1e9
    bpl = g["bytes"] / g["launches"]
    ratio = traffic_from_profiles("traffic_level_step_swirl_amr.json", nt)
    copy_gbs = stream_copy_gbs()
    l8 = None
    if not args.no_l8:
        u = uniform_workload(8, 32, args.l8_steps, args.l8_steps, nt, not args.no_per_level, seg)
        l8 = {"workload": u["config"]["workload"], "value": u["value"], "unit": "cell-updates/s",
              "ms_per_step": u["ms_per_step"], "roofline": u["roofline"],
              "per_level": u["per_level"], "fused_over_per_level": u["fused_over_per_level"]}
        torch.cuda.empty_cache()
    lv = w["leaves"][:, 0]
    per_level = res.get("per_level")
    out = {
        "metric": METRIC, "value": g["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warm, "ms_per_step": g["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"swirl_amr: adaptive levels 3-7, 32x32 patches, 2 ghost layers, FP64 scalar "
                               f"advection, swirl field T=1, seeded 8-Gaussian data (seed 3), multirate "
                               f"(31 level-steps per coarse step), regrid every 2 coarse steps by |grad q| > 0.05, "
                               f"{steps} coarse steps after {warm}",
                   "patches_start": len(lv), "patches_end": g["patches_end"], "mx": 32,
                   "mode": "fused: one ghost-gathering advance kernel per level-step, the coarse steps between "
                           "two regrids replayed from one hipGraph",
                   "threads_per_patch": nt, "sweep_segment_cells": seg, "cell_updates": g["cells"],
                   "regrid_ms_each": 1e3 * g["regrid_s"] / max(1, g["regrids"]),
                   "value_with_regrid": g["cells"] / (g["advance_s"] + g["regrid_s"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": (ratio * bpl) if ratio else None,
                     "kernel": level_step_name(32, nt, seg), "small_level_kernel": level_step_name(32, 512, 0),
                     "small_level_patches": "at most 4 per CU, on levels that are not complete", "launches": g["launches"],
                     "bytes_per_launch": bpl, "avg_launch_ms": 1e3 * g["advance_s"] / g["launches"],
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "per_level": per_level,
        "fused_over_per_level": (g["value"] / per_level["value"]) if per_level else None,
        "hbm_roofline_uniform_l8": l8,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(w),
    }
    print(json.dumps(out), flush=True)


def dam_break_workload(args):
    """Shallow-water dam break (levels 2-6, 16x16, reflecting walls), fixed
    coarse step, graph form against the per-level form, one JSON line."""
    import numpy as np
    import torch
    from paper_1703_03116_amd import binding as B
    from workloads import synth as S

    steps = args.steps if args.steps is not None else 100
    res = {}
    for mode in ("graph", "per_level"):
        w = S.workload("dam_break")
        ps = B.from_workload(w)
        if args.threads:
            ps.set_variant(args.threads)
            nt = args.threads
        else:
            nt = ps.autotune()
        lv = np.asarray(w["leaves"])[:, 0]
        dt = 0.6 / (w["mx"] << w["lmin"]) / 2.5   # finest-level Courant number <= 0.6 for speeds <= 2.5
        per_step = sum(int((lv == l).sum()) * w["mx"] ** 2 * (1 << (l - w["lmin"])) for l in np.unique(lv))
        ps.coarse_steps(dt, 2, mode)
        ps.prepare_steps(dt, steps, mode)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ps.coarse_steps(dt, steps, mode)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        ps.check()
        res[mode] = {"value": per_step * steps / sec, "ms_per_coarse_step": 1e3 * sec / steps,
                     "patches": len(lv)}
    out = {"metric": METRIC, "value": res["graph"]["value"], "unit": "cell-updates/s", "n_gpus": 1,
           "steps": steps, "warmup": 2, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "ms_per_step": res["graph"]["ms_per_coarse_step"],
           "dtype": "f64", "data": "synthetic", "config": {"workload": "dam_break", "threads_per_patch": nt},
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

    level, mx, n, every = 6, 32, (args.steps if args.steps is not None else 256), 16
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
