"""Host orchestration of dynamic adaptation (Sec. 4.1) around the GPU path.

Every ``regrid_every`` coarse steps: fill ghosts on all levels (tagging reads
neighbour differences), tag on the GPU (fc_tag_refine), adapt on the host
(fc_adapt: refine, coarsen complete sibling families, 2:1 balance), transfer
on the GPU (fc_regrid).  Between regrids the levels advance with multirate
subcycling through the fused persistent kernel.  Regridding is timed apart
from advance + fill, as the paper reports it separately.
"""
from __future__ import annotations

import time

import numpy as np
import torch


def regrid_once(store, tau_refine, tau_coarsen):
    """One tag/adapt/transfer cycle; returns the new leaf list (store order of
    the new mesh is its own; input order = the returned list)."""
    store.ghost_fill()
    tags, _ = store.tag(tau_refine, tau_coarsen)
    new = store.adapt(tags.cpu().numpy())
    store.regrid(new)
    return new


def run_adaptive(store, dt_coarse, ncoarse, regrid_every=2, tau_refine=0.05, tau_coarsen=None,
                 mode="graph", timings=None):
    """Advance ``ncoarse`` coarse steps with regridding every ``regrid_every``.

    Returns the number of cell updates performed (sum over level-steps of
    patches * mx^2).  ``timings`` (dict, optional) accumulates seconds of
    'advance' and 'regrid'.
    """
    tau_coarsen = 0.5 * tau_refine if tau_coarsen is None else tau_coarsen
    cells = 0
    done = 0
    while done < ncoarse:
        if done % regrid_every == 0 and done > 0:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            regrid_once(store, tau_refine, tau_coarsen)
            torch.cuda.synchronize()
            if timings is not None:
                timings["regrid"] = timings.get("regrid", 0.0) + time.perf_counter() - t0
        m = min(regrid_every - done % regrid_every, ncoarse - done)
        lv = store.leaves()[:, 0]
        per_step = sum(int((lv == l).sum()) * store.mx ** 2 * (1 << (int(l) - store.min_level))
                       for l in np.unique(lv))  # Python ints: a NumPy int32 would overflow over many steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        store.coarse_steps(dt_coarse, m, mode)
        torch.cuda.synchronize()
        if timings is not None:
            timings["advance"] = timings.get("advance", 0.0) + time.perf_counter() - t0
        cells += per_step * m
        done += m
    return cells
