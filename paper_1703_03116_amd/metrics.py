"""Host-side bookkeeping of the benchmark metric and the time-step rule."""
from __future__ import annotations


def cell_updates(level_counts, mx, lmin, time_stepping="multirate"):
    """Cell updates of one coarse step: sum over level-steps of P_l mx^2.

    Multirate: level l takes 2^(l - lmin) steps per coarse step; global
    stepping: every level takes one.  This is the paper's mx^2 * asteps
    (Table scale_rates counts patch advances "asteps").
    """
    tot = 0
    for l, p in level_counts.items():
        steps = (1 << (l - lmin)) if time_stepping == "multirate" else 1
        tot += p * mx * mx * steps
    return tot


def cell_update_rate(mx, patch_advances, seconds):
    """Cells advanced per second: mx^2 * asteps / wall (Sec. 5.1 tables)."""
    return mx * mx * patch_advances / seconds


def stable_dt(cfl, h, speed_max):
    """Fixed time step for a Courant number `cfl` on mesh width h: the
    paper's "dt = alpha dx" read with the advection speed (Sec. 5.1 prints
    final times consistent with dt = alpha dx / |u|)."""
    return cfl * h / speed_max
