"""Seeded synthetic inputs for the quadtree AMR advance + ghost-fill path.

This module is shared by the tests, the CPU oracle harness and the benchmark.
It holds only input recipes: quadtree leaf sets (pure geometry), seeded
parameters of initial fields and their point values at cell centres.  None of
the method's arithmetic (ghost filling, wave propagation, limiting, tagging,
time stepping) lives here.

Conventions
-----------
* The domain is the unit square, one block.  A leaf is ``(level, ix, iy)``
  with ``0 <= ix, iy < 2**level``; its quadrant is
  ``[ix, ix+1) x [iy, iy+1) * 2**-level``.
* A patch holds ``mx x mx`` interior cells; cell ``(i, j)`` of leaf
  ``(l, ix, iy)`` has centre ``((ix*mx + i + 0.5) h, (iy*mx + j + 0.5) h)``
  with ``h = 1 / (mx * 2**l)``.  Arrays are indexed ``[j][i]`` (x fastest).
* Interchange arrays of patch data are ``[nleaves][nfields][mx][mx]`` in the
  order of the leaf list they belong to.
* A brick is an ``nbx x nby`` arrangement of unit blocks.  In brick
  coordinates a leaf ``(l, ix, iy)`` has ``0 <= ix < nbx 2**l``,
  ``0 <= iy < nby 2**l`` and lies in block ``(ix >> l, iy >> l)``.  A block
  may carry an index orientation code 0..7 (bit 0 exchanges the two index
  directions, then bit 1 reverses the brick's first and bit 2 its second);
  leaves and patch data handed to a brick store are in the blocks' own
  indices (``brick_own_leaves``, ``brick_own_data``).
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# leaf sets
# --------------------------------------------------------------------------


def uniform_leaves(level: int, brick=(1, 1)) -> np.ndarray:
    """All quadrants of one level (``4**level`` per block), row-major in (iy, ix)."""
    n = 1 << level
    iy, ix = np.meshgrid(np.arange(n * brick[1]), np.arange(n * brick[0]), indexing="ij")
    lv = np.full(ix.size, level)
    return np.stack([lv, ix.ravel(), iy.ravel()], axis=1).astype(np.int32)


def refine_leaves(leaves, which) -> np.ndarray:
    """Replace every leaf whose index is in ``which`` by its four children."""
    which = set(int(k) for k in which)
    out = []
    for k, (l, ix, iy) in enumerate(np.asarray(leaves).tolist()):
        if k in which:
            for cy in (0, 1):
                for cx in (0, 1):
                    out.append((l + 1, 2 * ix + cx, 2 * iy + cy))
        else:
            out.append((l, ix, iy))
    return np.asarray(out, dtype=np.int32)


def hump_leaves() -> np.ndarray:
    """Levels 2-3 layout with refinement fixed around the centre.

    The sixteen level-2 quadrants tile the square; the four central ones,
    which cover [0.25, 0.75]^2, are refined once: 12 level-2 + 16 level-3
    leaves.
    """
    base = uniform_leaves(2)
    central = [k for k, (l, ix, iy) in enumerate(base.tolist())
               if ix in (1, 2) and iy in (1, 2)]
    return refine_leaves(base, central)


def _neighbour_offsets():
    return [(-1, 0), (1, 0), (0, -1), (0, 1), (-1, -1), (1, -1), (-1, 1), (1, 1)]


def balance_leaves(leaves, periodic=(True, True), brick=(1, 1)) -> np.ndarray:
    """Refine leaves until face- and corner-adjacent leaves differ by <= 1 level.

    A pure mesh-generation helper used to build input meshes.  Refinement
    only; the result is a 2:1 balanced leaf set covering the same square
    (brick, in brick coordinates).
    """
    cur = {tuple(x) for x in np.asarray(leaves).tolist()}
    while True:
        by_key = cur
        lmax = max(l for l, _, _ in cur)
        # finest-level coverage map: quadrant at lmax -> level of covering leaf
        nf = 1 << lmax
        nfx, nfy = nf * brick[0], nf * brick[1]
        cover = np.full((nfy, nfx), -1, dtype=np.int32)
        for l, ix, iy in by_key:
            s = 1 << (lmax - l)
            cover[iy * s:(iy + 1) * s, ix * s:(ix + 1) * s] = l
        to_refine = set()
        for l, ix, iy in by_key:
            s = 1 << (lmax - l)
            x0, y0 = ix * s, iy * s
            for dx, dy in _neighbour_offsets():
                # sample the finest-level quadrants just across the face/corner
                xs = [x0 - 1] if dx < 0 else ([x0 + s] if dx > 0 else range(x0, x0 + s))
                ys = [y0 - 1] if dy < 0 else ([y0 + s] if dy > 0 else range(y0, y0 + s))
                for yy in ys:
                    for xx in xs:
                        if not (0 <= xx < nfx):
                            if not periodic[0]:
                                continue
                            xx %= nfx
                        if not (0 <= yy < nfy):
                            if not periodic[1]:
                                continue
                            yy %= nfy
                        if cover[yy, xx] > l + 1:
                            to_refine.add((l, ix, iy))
        if not to_refine:
            break
        nxt = set()
        for leaf in cur:
            if leaf in to_refine:
                l, ix, iy = leaf
                for cy in (0, 1):
                    for cx in (0, 1):
                        nxt.add((l + 1, 2 * ix + cx, 2 * iy + cy))
            else:
                nxt.add(leaf)
        cur = nxt
    return np.asarray(sorted(cur), dtype=np.int32)


def refine_where(predicate, lmin: int, lmax: int, periodic=(True, True)) -> np.ndarray:
    """Start from uniform ``lmin`` and refine a leaf while ``predicate(leaf)``.

    ``predicate(level, ix, iy) -> bool`` is a geometric input rule (for
    example "the quadrant lies within a band around a feature").  The
    result is 2:1 balanced.
    """
    cur = [tuple(x) for x in uniform_leaves(lmin).tolist()]
    for _ in range(lmax - lmin):
        nxt = []
        for l, ix, iy in cur:
            if l < lmax and predicate(l, ix, iy):
                for cy in (0, 1):
                    for cx in (0, 1):
                        nxt.append((l + 1, 2 * ix + cx, 2 * iy + cy))
            else:
                nxt.append((l, ix, iy))
        cur = nxt
    return balance_leaves(np.asarray(cur, dtype=np.int32), periodic)


def random_balanced_leaves(seed: int, lmin: int, lmax: int, p_refine=0.35,
                           periodic=(True, True), brick=(1, 1)) -> np.ndarray:
    """Random 2:1 balanced leaf set spanning levels lmin..lmax (test meshes;
    brick coordinates for a brick)."""
    rng = np.random.default_rng(seed)
    cur = [tuple(x) for x in uniform_leaves(lmin, brick).tolist()]
    for _ in range(lmax - lmin):
        nxt = []
        for l, ix, iy in cur:
            if l < lmax and rng.random() < p_refine:
                for cy in (0, 1):
                    for cx in (0, 1):
                        nxt.append((l + 1, 2 * ix + cx, 2 * iy + cy))
            else:
                nxt.append((l, ix, iy))
        cur = nxt
    return balance_leaves(np.asarray(cur, dtype=np.int32), periodic, brick)


def replicate_leaves(leaves, brick) -> np.ndarray:
    """One block's leaf set copied into every block of a brick (brick
    coordinates, block-major): the replicated weak-scaling layout."""
    out = []
    for by in range(brick[1]):
        for bx in range(brick[0]):
            for l, ix, iy in np.asarray(leaves).tolist():
                out.append((l, ix + (bx << l), iy + (by << l)))
    return np.asarray(out, dtype=np.int32)


# --------------------------------------------------------------------------
# block orientations of a brick (input format conversion only)
# --------------------------------------------------------------------------


def own_to_brick_index(code: int, n: int, a, b):
    """Block-own index (a, b) -> brick index inside the block, n per side."""
    p, q = (b, a) if code & 1 else (a, b)
    x = n - 1 - p if code & 2 else p
    y = n - 1 - q if code & 4 else q
    return x, y


def brick_to_own_index(code: int, n: int, x, y):
    """Inverse of own_to_brick_index."""
    p = n - 1 - x if code & 2 else x
    q = n - 1 - y if code & 4 else y
    return (q, p) if code & 1 else (p, q)


def brick_own_leaves(leaves, brick, orient) -> np.ndarray:
    """Leaves in brick coordinates -> the blocks' own coordinates."""
    out = []
    for l, ix, iy in np.asarray(leaves).tolist():
        bx, by, n = ix >> l, iy >> l, 1 << l
        a, b = brick_to_own_index(int(orient[bx + brick[0] * by]), n, ix - bx * n, iy - by * n)
        out.append((l, bx * n + a, by * n + b))
    return np.asarray(out, dtype=np.int32)


def _leaf_code(leaf, brick, orient):
    l, ix, iy = (int(v) for v in leaf)
    return int(orient[(ix >> l) + brick[0] * (iy >> l)])


def brick_own_data(q, leaves, brick, orient, ghosts: int = 0) -> np.ndarray:
    """Patch arrays ``[n][F][M][M]`` laid out in brick directions -> the
    blocks' own index directions (M = mx + 2 ghosts; ghost cells map to
    ghost cells).  Leaves in brick coordinates, same order."""
    q = np.asarray(q)
    out = np.empty_like(q)
    M = q.shape[-1]
    a, b = np.meshgrid(np.arange(M) - ghosts, np.arange(M) - ghosts, indexing="xy")
    for k, leaf in enumerate(np.asarray(leaves)):
        x, y = own_to_brick_index(_leaf_code(leaf, brick, orient), M - 2 * ghosts, a, b)
        out[k] = q[k][..., y + ghosts, x + ghosts]
    return out


def brick_aligned_data(q, leaves, brick, orient, ghosts: int = 0) -> np.ndarray:
    """Inverse of brick_own_data."""
    q = np.asarray(q)
    out = np.empty_like(q)
    M = q.shape[-1]
    x, y = np.meshgrid(np.arange(M) - ghosts, np.arange(M) - ghosts, indexing="xy")
    for k, leaf in enumerate(np.asarray(leaves)):
        a, b = brick_to_own_index(_leaf_code(leaf, brick, orient), M - 2 * ghosts, x, y)
        out[k] = q[k][..., b + ghosts, a + ghosts]
    return out


# --------------------------------------------------------------------------
# cell geometry of a leaf
# --------------------------------------------------------------------------


def cell_centres(leaf, mx: int):
    """Cell-centre coordinates (x, y), each ``[mx][mx]`` indexed [j][i]."""
    l, ix, iy = (int(v) for v in leaf)
    h = 1.0 / (mx * (1 << l))
    i = np.arange(mx)
    xc = (ix * mx + i + 0.5) * h
    yc = (iy * mx + i + 0.5) * h
    x, y = np.meshgrid(xc, yc, indexing="xy")
    return x, y


def sample_on_leaves(fn, leaves, mx: int, nfields: int = 1) -> np.ndarray:
    """Evaluate ``fn(x, y) -> [nfields] arrays`` at every leaf's cell centres."""
    leaves = np.asarray(leaves)
    out = np.empty((len(leaves), nfields, mx, mx), dtype=np.float64)
    for k, leaf in enumerate(leaves):
        x, y = cell_centres(leaf, mx)
        v = fn(x, y)
        if nfields == 1 and not isinstance(v, (list, tuple)):
            v = [v]
        for f in range(nfields):
            out[k, f] = v[f]
    return out


# --------------------------------------------------------------------------
# initial fields
# --------------------------------------------------------------------------


def gaussian_params(seed: int, count: int = 8):
    """Seeded sum-of-Gaussians recipe: centres U[0.15,0.85]^2, widths
    U[0.02,0.1], amplitudes U[0.5,1]."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.15, 0.85, size=(count, 2))
    w = rng.uniform(0.02, 0.1, size=count)
    a = rng.uniform(0.5, 1.0, size=count)
    return {"c": c, "w": w, "a": a}


def gaussians(params):
    """q(x, y) = sum_k a_k exp(-|x - c_k|^2 / w_k^2) (no periodic images)."""
    c, w, a = params["c"], params["w"], params["a"]

    def fn(x, y):
        q = np.zeros_like(x)
        for k in range(len(a)):
            r2 = (x - c[k, 0]) ** 2 + (y - c[k, 1]) ** 2
            q = q + a[k] * np.exp(-r2 / (w[k] * w[k]))
        return q
    return fn


def gaussians_on_waves(params):
    """The Gaussian sum plus two periodic plane waves, so that cell
    differences vanish only near isolated curves (no flat regions where the
    Gaussians underflow): q = gaussians(params) + 0.25 sin(2 pi (x + 2y) +
    0.4) + 0.15 cos(2 pi (3x - y))."""
    g = gaussians(params)

    def f(x, y):
        return (g(x, y) + 0.25 * np.sin(2 * np.pi * (x + 2 * y) + 0.4)
                + 0.15 * np.cos(2 * np.pi * (3 * x - y)))
    return f


def gaussian_grad_max(params, leaf) -> float:
    """Upper bound of |grad q| over a leaf's quadrant (input-mesh rule)."""
    l, ix, iy = (int(v) for v in leaf)
    s = 1.0 / (1 << l)
    x0, y0 = ix * s, iy * s
    c, w, a = params["c"], params["w"], params["a"]
    g = 0.0
    for k in range(len(a)):
        # closest point of the quadrant to the centre, distance r; the
        # Gaussian's radial slope peaks at r = w/sqrt(2)
        dx = max(x0 - c[k, 0], 0.0, c[k, 0] - (x0 + s))
        dy = max(y0 - c[k, 1], 0.0, c[k, 1] - (y0 + s))
        r = np.hypot(dx, dy)
        rr = max(r, w[k] / np.sqrt(2.0)) if r <= w[k] / np.sqrt(2.0) else r
        g += a[k] * 2.0 * rr / (w[k] ** 2) * np.exp(-rr * rr / w[k] ** 2)
    return g


def hump(x, y):
    """The single Gaussian hump exp(-100 |x - (0.5, 0.5)|^2)."""
    return np.exp(-100.0 * ((x - 0.5) ** 2 + (y - 0.5) ** 2))


def dam_break_params(seed: int):
    rng = np.random.default_rng(seed)
    return {"c": rng.uniform(0.25, 0.75, size=2), "r": 0.2}


def dam_break(params):
    """h = 2 inside the circle, 1 outside; hu = hv = 0."""
    cx, cy = params["c"]
    r = params["r"]

    def fn(x, y):
        inside = (x - cx) ** 2 + (y - cy) ** 2 < r * r
        h = np.where(inside, 2.0, 1.0)
        return [h, np.zeros_like(x), np.zeros_like(x)]
    return fn


def smooth_directions(seed: int, count: int, leaves, mx: int):
    """Seeded smooth perturbation directions: random Gaussian sums with widths
    in [0.05, 0.2], scaled to max-abs 1."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = 6
        p = {"c": rng.uniform(0.0, 1.0, size=(k, 2)),
             "w": rng.uniform(0.05, 0.2, size=k),
             "a": rng.uniform(-1.0, 1.0, size=k)}
        d = sample_on_leaves(gaussians(p), leaves, mx)
        d /= np.abs(d).max()
        out.append(d)
    return out


# --------------------------------------------------------------------------
# the five named workloads
# --------------------------------------------------------------------------


def workload(name: str, **over):
    """Return a dict describing one synthetic workload.

    keys: leaves, mx, mbc, equation, velocity, vel_params, bc, q0, lmin,
    lmax, dt_coarse, steps, time_stepping, extra.
    """
    if name == "hump_l23":
        leaves = hump_leaves()
        mx = over.get("mx", 8)
        q0 = sample_on_leaves(hump, leaves, mx)
        dt = 0.9 / (mx * 4)            # level-2 cells, |u|max = 1
        w = dict(leaves=leaves, mx=mx, equation="advection",
                 velocity="constant", vel_params=(1.0, 0.5, 0.0),
                 bc=("periodic",) * 4, q0=q0, lmin=2, lmax=3,
                 dt_coarse=dt, steps=100, time_stepping="multirate")
    elif name.startswith("swirl_uniform"):
        level = over.get("level", 5)
        leaves = uniform_leaves(level)
        mx = over.get("mx", 32)
        seed = over.get("seed", 2)
        q0 = sample_on_leaves(gaussians(gaussian_params(seed)), leaves, mx)
        dt = 0.9 / (mx * (1 << level))
        w = dict(leaves=leaves, mx=mx, equation="advection",
                 velocity="swirl", vel_params=(1.0, 0.0, 0.0),
                 bc=("periodic",) * 4, q0=q0, lmin=level, lmax=level,
                 dt_coarse=dt, steps=over.get("steps", 500),
                 time_stepping="multirate")
    elif name == "swirl_amr":
        lmin, lmax = over.get("lmin", 3), over.get("lmax", 7)
        mx = over.get("mx", 32)
        seed = over.get("seed", 3)
        gp = gaussian_params(seed)
        tau = over.get("tau", 0.05)
        # geometric input rule: refine a quadrant while an analytic upper
        # bound of |grad q0| over it exceeds tau, then 2:1 balance
        leaves = refine_where(lambda l, ix, iy: gaussian_grad_max(gp, (l, ix, iy)) > tau, lmin, lmax)
        q0 = sample_on_leaves(gaussians(gp), leaves, mx)
        dt = 0.9 / (mx * (1 << lmin))
        w = dict(leaves=leaves, mx=mx, equation="advection",
                 velocity="swirl", vel_params=(1.0, 0.0, 0.0),
                 bc=("periodic",) * 4, q0=q0, lmin=lmin, lmax=lmax,
                 dt_coarse=dt, steps=over.get("steps", 40),
                 time_stepping="multirate")
    elif name == "dam_break":
        lmin, lmax = over.get("lmin", 2), over.get("lmax", 6)
        mx = over.get("mx", 16)
        dp = dam_break_params(over.get("seed", 4))
        cx, cy = dp["c"]

        def near_edge(l, ix, iy):
            s = 1.0 / (1 << l)
            qx, qy = (ix + 0.5) * s, (iy + 0.5) * s
            d = abs(np.hypot(qx - cx, qy - cy) - dp["r"])
            return d < 0.75 * s + 0.02

        leaves = refine_where(near_edge, lmin, lmax, periodic=(False, False))
        q0 = sample_on_leaves(dam_break(dp), leaves, mx, nfields=3)
        w = dict(leaves=leaves, mx=mx, equation="swe", gravity=1.0,
                 velocity="none", vel_params=(0.0, 0.0, 0.0),
                 bc=("reflect",) * 4, q0=q0, lmin=lmin, lmax=lmax,
                 dt_coarse=None, steps=over.get("steps", 20),
                 time_stepping="multirate")
    else:
        raise KeyError(name)
    w["mbc"] = 2
    w["name"] = name
    return w
