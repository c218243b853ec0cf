"""Host orchestration of dynamic adaptation (Sec. 4.1) around the GPU path.

Every ``regrid_every`` coarse steps: fill ghosts on all levels (tagging reads
neighbour differences), tag on the GPU (fc_tag_refine), adapt on the host
(fc_adapt: refine, coarsen complete sibling families, 2:1 balance), transfer
on the GPU (fc_regrid).  Between regrids the levels advance with multirate
subcycling in the chosen execution form.  Regridding, and the graph capture a
new mesh needs, are timed apart from advance + fill, as the paper reports
regridding separately.
"""
from __future__ import annotations

import time

import numpy as np
import torch


def regrid_once(store, tau_refine, tau_coarsen, smooth=False, device=True):
    """One tag/adapt/transfer cycle; returns the new leaf list (store order of
    the new mesh is its own; input order = the returned list).  device: the
    adaptation runs on the GPU (fc_adapt_device; only the new leaf list comes
    to the host), else on the host (fc_adapt); smooth: smooth refinement."""
    store.ghost_fill()
    tags, _ = store.tag(tau_refine, tau_coarsen)
    new = store.adapt_device(tags, smooth) if device else store.adapt(tags.cpu().numpy(), smooth)
    store.regrid(new)
    return new


def step_counts(store):
    """Per coarse step of the current mesh: cell updates (sum over level-steps
    of patches * mx^2), level-step launches of the fused forms, and the
    algorithmic bytes of those launches (each patch reads its tile with halo
    once and writes its interior once)."""
    lv = store.leaves()[:, 0]
    cells = launches = nbytes = 0
    for l in np.unique(lv):
        p, k = int((lv == l).sum()), 1 << (int(l) - store.min_level)
        cells += p * store.mx ** 2 * k      # Python ints: NumPy int32 would wrap over many steps
        launches += k
        nbytes += p * store.F * 8 * (store.N ** 2 + store.mx ** 2) * k
    return cells, launches, nbytes


def run_adaptive(store, dt_coarse, ncoarse, regrid_every=2, tau_refine=0.05, tau_coarsen=None,
                 mode="graph", timings=None, smooth=False, device_adapt=True):
    """Advance ``ncoarse`` coarse steps with regridding every ``regrid_every``.

    Returns the number of cell updates performed.  smooth / device_adapt as
    in regrid_once.  ``timings`` (dict,
    optional) accumulates 'advance' (seconds of advance + fill, HIP events on
    the stream the work runs on), 'regrid' (seconds of tag + adapt + transfer
    + the graph capture for the new mesh), 'launches' and 'bytes' (level-step
    launches and their algorithmic bytes) and 'regrids'.
    """
    tau_coarsen = 0.5 * tau_refine if tau_coarsen is None else tau_coarsen
    stream = torch.cuda.current_stream()
    events = []
    cells = 0
    done = 0
    tm = timings if timings is not None else {}
    for k in ("advance", "regrid", "launches", "bytes", "regrids"):
        tm.setdefault(k, 0)
    while done < ncoarse:
        m = min(regrid_every - done % regrid_every, ncoarse - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if done % regrid_every == 0 and done > 0:
            regrid_once(store, tau_refine, tau_coarsen, smooth, device_adapt)
            tm["regrids"] += 1
        store.prepare_steps(dt_coarse, m, mode)
        torch.cuda.synchronize()
        tm["regrid"] += time.perf_counter() - t0
        c, nl, nb = step_counts(store)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        store.coarse_steps(dt_coarse, m, mode)
        e1.record(stream)
        events.append((e0, e1))
        cells += c * m
        tm["launches"] += nl * m
        tm["bytes"] += nb * m
        done += m
    torch.cuda.synchronize()
    tm["advance"] += sum(a.elapsed_time(b) for a, b in events) / 1e3
    return cells
