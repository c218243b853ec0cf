"""More pins of the FP64 CPU oracle: the parts a single-velocity or 1-D test
cannot see.

* Edge velocities of the swirl field against the stream function's exact
  edge differences in 40-digit arithmetic (Sec. 5.1 defines the velocity by a
  stream function, u = psi_y, v = -psi_x).
* Corner transport under a variable velocity: the one-step response of the
  first-order unsplit scheme to a unit cell, in closed form.
* Mirror symmetry of the swirl step (the field flips sign under a mirror,
  and cos(pi (t + 1)) = -cos(pi t) flips it back).
* Flow reversal: cos(pi t / T) turns the swirl around at T/2, so the exact
  solution at T equals q0; the scheme converges to it at second order.
* Coarse-to-fine ghost interpolation itself (eq. ghost_fine, "monotone",
  Sec. 4.1): bounded by the coarse 5-point stencil and averaging back to the
  coarse value, on random 2:1 meshes.
* Shallow-water transverse splitting: a smooth simple wave travelling along
  the diagonal, against its exact solution by characteristics.
* Shallow-water entropy fix: transonic rarefactions against the exact
  Riemann solution, with no stationary expansion shock at the sonic point.

Each case fails for a plausible mistake in the part it pins (for example a
velocity taken at the wrong edge or time, sigma dropped, an unlimited
interpolation slope, transverse waves dropped or sent the wrong way, the
entropy fix switched off).
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from workloads import synth as S


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def to_global(leaves, arr, mx, f=0):
    leaves = np.asarray(leaves)
    n = mx << int(leaves[0, 0])
    G = np.zeros((n, n))
    for k, (l, ix, iy) in enumerate(leaves):
        G[iy * mx:(iy + 1) * mx, ix * mx:(ix + 1) * mx] = arr[k, f]
    return G


def from_global(leaves, G, mx, nf=1):
    out = np.zeros((len(leaves), nf, mx, mx))
    for k, (l, ix, iy) in enumerate(np.asarray(leaves)):
        for f in range(nf):
            Gf = G[f] if nf > 1 else G
            out[k, f] = Gf[iy * mx:(iy + 1) * mx, ix * mx:(ix + 1) * mx]
    return out


# ---------------------------------------------------------------------------
# swirl velocities
# ---------------------------------------------------------------------------

def _psi(x, y, t, T=1):
    import mpmath as mp
    return mp.sin(mp.pi * x) ** 2 * mp.sin(mp.pi * y) ** 2 * mp.cos(mp.pi * t / T) / mp.pi


@pytest.mark.parametrize("level,mx", [(0, 8), (3, 16)])
def test_swirl_edge_velocities_are_stream_function_differences(O, level, mx):
    """u on an x-edge is the mean of psi_y along the edge, (psi(top) -
    psi(bottom)) / h, and v on a y-edge is -(psi(right) - psi(left)) / h,
    with psi = sin^2(pi x) sin^2(pi y) cos(pi t / T) / pi; both evaluated in
    40-digit arithmetic.  Fixes the signs (u = psi_y, v = -psi_x), the edge
    and cell indexing and the sin(pi h)/(pi h) edge-average factor."""
    import mpmath as mp
    mp.mp.dps = 40
    o = O.Oracle(S.uniform_leaves(level), mx=mx, velocity="swirl", vel_params=(1.0, 0, 0))
    n = mx << level
    h = mp.mpf(1) / n
    rng = np.random.default_rng(level)
    worst = 0.0
    for _ in range(60):
        I, J = int(rng.integers(0, n + 1)), int(rng.integers(0, n))
        tm = float(rng.uniform(0, 1))
        u_ex = (_psi(I * h, (J + 1) * h, tm) - _psi(I * h, J * h, tm)) / h
        v_ex = -(_psi((J + 1) * h, I * h, tm) - _psi(J * h, I * h, tm)) / h  # column J, y-edge I
        u = o.edge_velocity(level, 0, I % n, J, tm)
        v = o.edge_velocity(level, 1, J, I % n, tm)
        worst = max(worst, abs(u - float(u_ex)), abs(v - float(v_ex)))
    assert worst < 1e-14, worst


# ---------------------------------------------------------------------------
# corner transport under a variable velocity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cell", [(5, 2), (2, 2), (2, 5), (5, 5), (6, 1)])
def test_corner_transport_of_a_unit_cell(O, cell):
    """First-order unsplit step (no limiter correction) from a single unit
    cell on one periodic 8x8 patch in the swirl field.  The unit moves into
    the diagonal neighbour (i+sx, j+sy), sx, sy the signs of the velocities
    around it, along two paths: across the x-edge and then up or down with
    the v of the cell it entered, or across the y-edge and then sideways
    with the u of the cell it entered (corner transport upwind).  In closed
    form the diagonal neighbour receives
        1/2 lam^2 (|u(xe, j)| |v(i+sx, ye)| + |v(i, ye)| |u(xe, j+sy)|),
    velocities at the mid-step time; the other three diagonal neighbours
    receive nothing.  A velocity taken at the wrong edge, cell or time, or a
    transverse wave sent the wrong way, changes these numbers."""
    import mpmath as mp
    mp.mp.dps = 40
    mx, level = 8, 0
    i0, j0 = cell
    t, dt = 0.13, 0.05
    tm = t + 0.5 * dt
    lam = dt * mx
    o = O.Oracle([[0, 0, 0]], mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter="first")
    h = mp.mpf(1) / mx

    def u(I, J):   # x-edge I, row J (periodic)
        I, J = I % mx, J % mx
        return float((_psi(I * h, (J + 1) * h, tm) - _psi(I * h, J * h, tm)) / h)

    def v(I, J):   # column I, y-edge J
        I, J = I % mx, J % mx
        return float(-(_psi((I + 1) * h, J * h, tm) - _psi(I * h, J * h, tm)) / h)

    sx = 1 if u(i0 + 1, j0) > 0 else -1
    sy = 1 if v(i0, j0 + 1) > 0 else -1
    xe = i0 + 1 if sx > 0 else i0          # the x-edge the unit leaves through
    ye = j0 + 1 if sy > 0 else j0
    # the case is clean only if every velocity on the two paths points the same way
    assert np.sign(u(xe, j0)) == sx and np.sign(u(xe, j0 + sy)) == sx
    assert np.sign(v(i0, ye)) == sy and np.sign(v(i0 + sx, ye)) == sy
    q = np.zeros((1, 1, mx, mx))
    q[0, 0, j0, i0] = 1.0
    o.set_interior(q)
    o.ghost_fill()
    o.advance_level(0, t, dt)
    r = o.interior()[0, 0]
    want = 0.5 * lam * lam * (abs(u(xe, j0)) * abs(v(i0 + sx, ye)) + abs(v(i0, ye)) * abs(u(xe, j0 + sy)))
    assert want > 1e-3
    assert abs(r[(j0 + sy) % mx, (i0 + sx) % mx] - want) < 1e-14, (r[(j0 + sy) % mx, (i0 + sx) % mx], want)
    for ax, ay in ((-sx, sy), (sx, -sy), (-sx, -sy)):
        assert abs(r[(j0 + ay) % mx, (i0 + ax) % mx]) < 1e-17


# ---------------------------------------------------------------------------
# mirror symmetry and flow reversal of the swirl
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("limiter", ["mc", "lw"])
@pytest.mark.parametrize("axis", [0, 1])
def test_swirl_mirror_symmetry(O, limiter, axis):
    """Mirroring x -> 1 - x (or y -> 1 - y) negates the swirl field, and
    c(t + 1) = cos(pi (t + 1)) = -c(t) negates it back: the mirrored data
    started one period of c later evolve into the mirror image of the
    original run (to rounding), through every edge, limiter and transverse
    term of the step."""
    L = S.uniform_leaves(2)
    mx = 8
    rng = np.random.default_rng(11 + axis)
    G = S.gaussians(S.gaussian_params(3))
    q = S.sample_on_leaves(G, L, mx) + 0.05 * rng.random((16, 1, mx, mx))
    Gq = to_global(L, q, mx)
    Gm = Gq[:, ::-1] if axis == 0 else Gq[::-1, :]
    a = O.Oracle(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter=limiter)
    b = O.Oracle(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter=limiter)
    a.set_interior(q)
    b.set_interior(from_global(L, np.ascontiguousarray(Gm), mx))
    dt = 0.9 / 32
    t = 0.07
    for s in range(10):
        a.coarse_step(t + s * dt, dt)
        b.coarse_step(t + 1.0 + s * dt, dt)
    A, Bm = to_global(L, a.interior(), mx), to_global(L, b.interior(), mx)
    Bm = Bm[:, ::-1] if axis == 0 else Bm[::-1, :]
    assert np.abs(A - Bm).max() < 1e-13


@pytest.mark.parametrize("limiter,min_order", [("lw", 1.9), ("mc", 1.75)])
def test_swirl_reversal_converges_at_second_order(O, limiter, min_order):
    """With c(t) = cos(pi t / T) the flow turns around at T/2 and the exact
    solution at T = 1 is q0 itself.  Halving h must cut the L1 error by
    about four: a first-order time error (velocities at t instead of the
    mid-step time) or a first-order space error does not."""
    errs = []
    for lev in (3, 4, 5):
        L = S.uniform_leaves(lev)
        mx = 8
        q0 = S.sample_on_leaves(lambda x, y: np.exp(-((x - 0.5) ** 2 + (y - 0.72) ** 2) / 0.12 ** 2), L, mx)
        o = O.Oracle(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter=limiter)
        o.set_interior(q0)
        n = mx << lev
        nst = int(np.ceil(1.0 / (0.9 / n)))
        dt = 1.0 / nst
        for s in range(nst):
            o.coarse_step(s * dt, dt)
        errs.append(np.abs(o.interior() - q0).sum() / n / n)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders.min() > min_order, (errs, orders)


# ---------------------------------------------------------------------------
# coarse-to-fine ghost interpolation
# ---------------------------------------------------------------------------

def _covering(leafset, l, I, J, mx):
    """Level and coordinates of the leaf containing the centre of level-l
    cell (I, J): the level-l quadrant, its parent or one of its children."""
    for cand in ((l, I // mx, J // mx), (l - 1, (I // mx) >> 1, (J // mx) >> 1),
                 (l + 1, (2 * I) // mx, (2 * J) // mx)):
        if cand in leafset:
            return cand
    return None


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("bc", ["periodic", "reflect"])
def test_fine_ghost_interpolation_bounded_and_conservative(O, seed, bc):
    """Every fine ghost cell filled from a coarser neighbour (eq. ghost_fine)
    lies within [min, max] of the coarse cell's 5-point stencil (the
    "monotone" interpolation of Sec. 4.1), and the four fine ghost cells
    covering one coarse cell average back to it (the +-1 direction vectors
    cancel).  Random data on random 2:1 meshes; the coarse stencil is read
    from the coarse patch after the fill (its own ghosts included)."""
    per = bc == "periodic"
    L = S.random_balanced_leaves(20 + seed, 2, 5, periodic=(per, per))
    mx, m = 8, 2
    eq = "advection" if per else "swe"
    o = O.Oracle(L, mx=mx, equation=eq, bc=(bc,) * 4, velocity="constant" if per else "none")
    rng = np.random.default_rng(seed)
    F = o.F
    o.set_interior(1.0 + rng.random((len(L), F, mx, mx)))
    o.ghost_fill()
    full = o.full()
    idx = {tuple(x): k for k, x in enumerate(L.tolist())}
    checked = 0
    groups = {}
    for k, (l, ix, iy) in enumerate(L.tolist()):
        nl = mx << l
        for j in range(-m, mx + m):
            for i in range(-m, mx + m):
                if 0 <= i < mx and 0 <= j < mx:
                    continue
                I, J = ix * mx + i, iy * mx + j
                if not (0 <= I < nl and 0 <= J < nl):
                    if not per:
                        continue
                    I, J = I % nl, J % nl
                cov = _covering(idx, l, I, J, mx)
                assert cov is not None
                if cov[0] != l - 1:
                    continue
                kc = idx[cov]
                ic, jc = I // 2 - cov[1] * mx, J // 2 - cov[2] * mx
                for f in range(F):
                    P = full[kc, f]
                    st = [P[jc + m, ic + m], P[jc + m, ic + m - 1], P[jc + m, ic + m + 1],
                          P[jc + m - 1, ic + m], P[jc + m + 1, ic + m]]
                    g = full[k, f, j + m, i + m]
                    assert min(st) - 1e-15 <= g <= max(st) + 1e-15, (k, i, j, f, g, st)
                    groups.setdefault((k, f, (i + m) // 2, (j + m) // 2), []).append((g, st[0]))
                checked += 1
    assert checked > 200
    full_groups = 0
    for vals in groups.values():
        if len(vals) == 4:
            assert abs(sum(v for v, _ in vals) / 4 - vals[0][1]) < 1e-15
            full_groups += 1
    assert full_groups > 50


# ---------------------------------------------------------------------------
# shallow water: diagonal simple wave (transverse splitting)
# ---------------------------------------------------------------------------

def _simple_wave(s, t, hbar=1.0, a=0.1, g=1.0):
    """Exact right-going simple wave along n = (1, 1)/sqrt(2), as a function
    of s = x + y (period 1).  The Riemann invariant u_n - 2c is -2 c_bar
    everywhere, u_n + c = 3c - 2 c_bar is carried along straight
    characteristics, so h(s, t) = h0(s0) with s = s0 + sqrt(2) (3 c(s0) - 2
    c_bar) t (before the wave breaks).  Returns h, u_n."""
    cb = np.sqrt(g * hbar)
    h0 = lambda z: hbar + a * np.sin(2 * np.pi * z)
    spd = lambda z: np.sqrt(2.0) * (3 * np.sqrt(g * h0(z)) - 2 * cb)
    s0 = s - spd(s) * t
    for _ in range(60):   # Newton on s0 + spd(s0) t - s = 0 (monotone before breaking)
        dh = a * 2 * np.pi * np.cos(2 * np.pi * s0)
        dsp = np.sqrt(2.0) * 3 * g * dh / (2 * np.sqrt(g * h0(s0)))
        s0 = s0 - (s0 + spd(s0) * t - s) / (1 + dsp * t)
    h = h0(s0)
    return h, 2 * (np.sqrt(g * h) - cb)


@pytest.mark.parametrize("limiter,min_order", [("lw", 1.85), ("mc", 1.6)])
def test_swe_diagonal_simple_wave_converges(O, limiter, min_order):
    """A smooth simple wave moving along the diagonal on the periodic
    square, at a Courant number of 0.8 per direction (their sum exceeds 1:
    the unsplit scheme is stable there only with its transverse terms).
    The error against the exact solution falls at second order; dropping
    the transverse splitting, or sending its up- and down-going parts the
    wrong way, leaves a first-order cross-derivative error or instability."""
    T = 0.2
    errs = []
    for lev in (2, 3, 4):
        L = S.uniform_leaves(lev)
        mx = 8
        n = mx << lev

        def init(x, y):
            h, un = _simple_wave(x + y, 0.0)
            m = h * un / np.sqrt(2.0)
            return [h, m, m]
        q0 = S.sample_on_leaves(init, L, mx, nfields=3)
        o = O.Oracle(L, mx=mx, equation="swe", limiter=limiter, bc=("periodic",) * 4, velocity="none")
        o.set_interior(q0)
        smax = 1.2    # |u_n|/sqrt(2) + c stays below 1.12 for a = 0.1
        nst = int(np.ceil(T / (0.8 / n / smax)))
        dt = T / nst
        cfl = 0.0
        for s in range(nst):
            cfl = max(cfl, o.coarse_step(s * dt, dt))
        assert 0.7 < cfl < 0.8
        x = (np.arange(n) + 0.5) / n
        X, Y = np.meshgrid(x, x, indexing="xy")
        h_ex, un_ex = _simple_wave(X + Y, T)
        H = to_global(L, o.interior(), mx, 0)
        HU = to_global(L, o.interior(), mx, 1)
        e = np.abs(H - h_ex).sum() / n / n + np.abs(HU - h_ex * un_ex / np.sqrt(2.0)).sum() / n / n
        errs.append(e)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders.min() > min_order, (errs, orders)


# ---------------------------------------------------------------------------
# shallow water: transonic rarefactions (Harten-Hyman entropy fix)
# ---------------------------------------------------------------------------

def _riemann_rarefaction_shock(xi, hl, hr, g=1.0):
    """Exact solution of the dam break hl > hr at rest: a 1-rarefaction
    into the middle state, then a 2-shock (Stoker).  xi = (x - x0) / t.
    Returns h and u."""
    cl = np.sqrt(g * hl)

    def res(hm):
        return 2 * (cl - np.sqrt(g * hm)) - (hm - hr) * np.sqrt(0.5 * g * (1 / hm + 1 / hr))
    hm = brentq(res, hr, hl)
    um = 2 * (cl - np.sqrt(g * hm))
    s = hm * um / (hm - hr)
    h = np.full_like(xi, hl)
    u = np.zeros_like(xi)
    fan = (xi >= -cl) & (xi < um - np.sqrt(g * hm))
    h = np.where(fan, (2 * cl - xi) ** 2 / (9 * g), h)
    u = np.where(fan, 2 * (cl + xi) / 3, u)
    mid = (xi >= um - np.sqrt(g * hm)) & (xi < s)
    h = np.where(mid, hm, h)
    u = np.where(mid, um, u)
    h = np.where(xi >= s, hr, h)
    u = np.where(xi >= s, 0.0, u)
    return h, u, um - np.sqrt(g * hm)


def transonic_run(O, lev, mirrored, hr=0.05, limiter="mc", T=0.12):
    """The dam break h = 1 | h_r (or its mirror) along x on level `lev`
    (mx = 8, walls), run to T; returns the oracle, xi = (x - 1/2) / t (its
    sign flipped for mirrored data), h and the exact h."""
    L = S.uniform_leaves(lev)
    mx = 8
    n = mx << lev
    hl = 1.0

    def init(x, y):
        h = np.where(x < 0.5, hl, hr) if not mirrored else np.where(x < 0.5, hr, hl)
        return [h, 0 * x, 0 * x]
    o = O.Oracle(L, mx=mx, equation="swe", limiter=limiter, bc=("reflect",) * 4, velocity="none")
    o.set_interior(S.sample_on_leaves(init, L, mx, nfields=3))
    dt = 0.5 / n / 1.6
    nst = int(round(T / dt))
    for s in range(nst):
        o.coarse_step(s * dt, dt)
    x = (np.arange(n) + 0.5) / n
    xi = (x - 0.5) / (nst * dt)
    if mirrored:
        xi = -xi
    h_ex, _, tail = _riemann_rarefaction_shock(xi, hl, hr)
    H = to_global(L, o.interior(), mx, 0)
    return o, xi, H, h_ex, tail


@pytest.mark.parametrize("hr", [0.05, 0.01])
@pytest.mark.parametrize("mirrored", [False, True])
def test_swe_transonic_rarefaction_has_no_expansion_shock(O, mirrored, hr):
    """h = 1 next to a shallow h_r at rest: the 1-rarefaction (the
    3-rarefaction for the mirrored data) spans zero speed (its tail moves at
    u* - c* > 0).  The Roe solver alone keeps a stationary expansion shock at
    the sonic point, whose jump does not shrink under refinement (about 0.17
    for h_r = 0.05 with the first-order scheme).  With the entropy fix the
    first-order solution converges to the exact one and inside the fan no two
    neighbouring cells differ by more than three times the exact slope times
    h at the finest level.  First order: the limited second-order correction
    alone already smears the expansion shock, so only the first-order scheme
    shows what the Riemann solver does."""
    errs, jumps = [], []
    for lev in (3, 4, 5):
        o, xi, H, h_ex, tail = transonic_run(O, lev, mirrored, hr=hr, limiter="first")
        assert tail > 0.3                       # the fan really straddles xi = 0
        n = len(xi)
        row = H[n // 2]
        assert np.abs(H - row[None, :]).max() < 1e-13   # 1-D: every row the same
        errs.append(np.abs(row - h_ex).sum() / n)
        fan = (np.abs(xi) < 0.25)               # cells around the sonic point
        jumps.append(np.abs(np.diff(row))[fan[1:] & fan[:-1]].max())
    # exact slope of h in the fan near xi = 0: 4 c_l / (9 g t) per unit x
    assert jumps[-1] < 3 * (4 / 9 / 0.12) / (8 << 5) and jumps[-1] < 0.6 * jumps[0], jumps
    assert errs[0] / errs[1] > 1.4 and errs[1] / errs[2] > 1.4 and errs[-1] < 5.5e-3, errs


@pytest.mark.parametrize("mirrored", [False, True])
def test_swe_transonic_rarefaction_converges_mc(O, mirrored):
    """The same transonic dam break with the MC-limited scheme converges to
    the exact solution (L1 error halves with h)."""
    errs = []
    for lev in (3, 4, 5):
        o, xi, H, h_ex, tail = transonic_run(O, lev, mirrored, hr=0.05, limiter="mc")
        n = len(xi)
        errs.append(np.abs(H[n // 2] - h_ex).sum() / n)
    assert errs[0] / errs[1] > 1.8 and errs[1] / errs[2] > 1.8 and errs[-1] < 1.5e-3, errs
