"""Pins of the oracle's multiblock brick (Sec. 2.3, index transforms).

A brick is an nbx x nby arrangement of unit blocks, each a quadtree with its
own index orientation (one of the eight maps whose matrix A in eq. transform
is diagonal or anti-diagonal with entries +-1).  The oracle carries every
ghost index into the neighbour's own indices; nothing else in the method
changes.  What pins that:

* exact solutions that hold in any orientation: at Courant number one the
  scheme moves data exactly one cell per step, and with one velocity
  component zero every brick row follows the textbook 1-D scheme;
* the special case that reduces to the pinned one-block path: an aligned
  brick whose blocks all hold the same mesh and data (the paper's replicated
  weak-scaling layout, Sec. 5.1) reproduces the one-block periodic result bit
  for bit in every block;
* invariance: a brick of rotated and reflected blocks gives the aligned
  brick's result in each block's own indices.  Copies and interpolations
  (eq. ghost_fine is odd in d_k and in the one-sided differences) are bit
  for bit; averages (eq. ghost_coarse sums the four fine cells in the order
  of the coarse patch's d_k) and the update agree up to rounding order;
* mesh rules across block boundaries: 2:1 balance and tiling checked in the
  brick's geometry, adaptation (Sec. 4.1, 4.2) and transfer agree with the
  aligned brick.
"""
import numpy as np
import pytest

from workloads import synth as S

BR = (3, 2)                      # not square: the two brick directions cannot be confused
ALL8 = (4, 2)                    # eight blocks, one per orientation code


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def oriented(O, leaves, brick, orient, **kw):
    """Oracle on a brick whose leaves are given in brick coordinates."""
    own = S.brick_own_leaves(leaves, brick, orient)
    return O.Oracle(own, brick=brick, orient=orient, **kw)


def brick_field(leaves, q, mx, brick):
    """Uniform-level patches (brick coordinates, brick directions) -> one array."""
    l = int(leaves[0][0])
    G = np.zeros((brick[1] * mx << l, brick[0] * mx << l))
    for (lv, ix, iy), p in zip(np.asarray(leaves).tolist(), q):
        G[iy * mx:(iy + 1) * mx, ix * mx:(ix + 1) * mx] = p[0]
    return G


def from_brick_field(leaves, G, mx):
    out = np.empty((len(leaves), 1, mx, mx))
    for k, (l, ix, iy) in enumerate(np.asarray(leaves).tolist()):
        out[k, 0] = G[iy * mx:(iy + 1) * mx, ix * mx:(ix + 1) * mx]
    return out


def codes(seed, brick):
    return list(np.random.default_rng(seed).integers(0, 8, brick[0] * brick[1]))


# ---------------------------------------------------------------------------
# exact solutions in every orientation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("vel", [(1.0, 1.0), (-1.0, 1.0), (1.0, -1.0)])
def test_unit_courant_shift_every_orientation(O, vel):
    """u = (+-1, +-1) at Courant number one moves every cell one cell
    diagonally, across block faces and corners of all eight orientations."""
    mx, l = 8, 1
    L = S.uniform_leaves(l, ALL8)
    orient = list(range(8))
    rng = np.random.default_rng(1)
    G0 = rng.random((ALL8[1] * mx << l, ALL8[0] * mx << l))
    o = oriented(O, L, ALL8, orient, mx=mx, velocity="constant", vel_params=(vel[0], vel[1], 0.0))
    o.set_interior(S.brick_own_data(from_brick_field(L, G0, mx), L, ALL8, orient))
    h = 1.0 / (mx << l)
    for s in range(3):
        o.ghost_fill()
        o.advance_level(l, s * h, h)
    G = brick_field(L, S.brick_aligned_data(o.interior(), L, ALL8, orient), mx, ALL8)
    ref = np.roll(np.roll(G0, 3 * int(vel[1]), 0), 3 * int(vel[0]), 1)
    assert np.abs(G - ref).max() < 1e-15


def _textbook_1d(q, nu):
    """1-D high-resolution wave propagation, u > 0, MC limiter (LeVeque 2002,
    Ch. 6), periodic array."""
    W = q - np.roll(q, 1)
    Wup = np.roll(W, 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        th = np.where(W != 0, Wup / np.where(W != 0, W, 1.0), 0.0)
    phi = np.maximum(0.0, np.minimum(np.minimum((1 + th) / 2, 2.0), 2 * th))
    Wt = np.where(W != 0, phi * W, 0.0)
    return q - nu * W - 0.5 * nu * (1 - nu) * (np.roll(Wt, -1) - Wt)


@pytest.mark.parametrize("axis", [0, 1])
def test_one_dimensional_reduction_every_orientation(O, axis):
    """With one brick velocity component zero, every brick row (column)
    evolves by the textbook 1-D scheme, whatever each block's orientation
    (in a transposed block the brick's x-velocity is the block's second
    component, and transverse terms still vanish)."""
    mx, l = 8, 1
    L = S.uniform_leaves(l, ALL8)
    orient = [3, 6, 1, 4, 7, 0, 5, 2]
    rng = np.random.default_rng(7 + axis)
    G = rng.random((ALL8[1] * mx << l, ALL8[0] * mx << l))
    vp = (0.7, 0.0, 0.0) if axis == 0 else (0.0, 0.7, 0.0)
    o = oriented(O, L, ALL8, orient, mx=mx, velocity="constant", vel_params=vp)
    o.set_interior(S.brick_own_data(from_brick_field(L, G, mx), L, ALL8, orient))
    dt = 0.9 / (mx << l) / 0.7
    ref = G.copy()
    for s in range(5):
        o.ghost_fill()
        cfl = o.advance_level(l, s * dt, dt)
        assert abs(cfl - 0.9) < 1e-15
        if axis == 0:
            ref = np.stack([_textbook_1d(r, 0.9) for r in ref])
        else:
            ref = np.stack([_textbook_1d(c, 0.9) for c in ref.T]).T
    out = brick_field(L, S.brick_aligned_data(o.interior(), L, ALL8, orient), mx, ALL8)
    assert np.abs(out - ref).max() < 1e-14


# ---------------------------------------------------------------------------
# the replicated layout reduces to one periodic block
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_aligned_replicated_brick_equals_one_block(O, seed):
    """Sec. 5.1's replicated domain: the same mesh and data in every block
    of an aligned, periodic brick at u = (0.5, 0.5) is the one-block periodic
    problem in each block, bit for bit (fill, then multirate steps)."""
    mx = 8
    one = S.random_balanced_leaves(seed, 2, 4)
    rng = np.random.default_rng(seed)
    q = rng.random((len(one), 1, mx, mx))
    kw = dict(mx=mx, velocity="constant", vel_params=(0.5, 0.5, 0.0), lmin=2, lmax=4)
    a = O.Oracle(one, **kw)
    a.set_interior(q)
    Lb = S.replicate_leaves(one, BR)
    b = O.Oracle(Lb, brick=BR, **kw)
    b.set_interior(np.concatenate([q] * (BR[0] * BR[1])))
    a.ghost_fill()
    b.ghost_fill()
    nb = BR[0] * BR[1]
    assert np.array_equal(b.full(), np.concatenate([a.full()] * nb))
    dt = 0.8 / (mx << 2)
    for s in range(3):
        ca = a.coarse_step(s * dt, dt)
        cb = b.coarse_step(s * dt, dt)
        assert ca == cb
    assert np.array_equal(b.interior(), np.concatenate([a.interior()] * nb))


# ---------------------------------------------------------------------------
# rotated and reflected blocks give the rotated result
# ---------------------------------------------------------------------------

def _leaf_at(leaves):
    """Point location on a brick-coordinate leaf set: level-l cell (I, J) of
    mx-cell patches -> index of the leaf covering its centre."""
    d = {(l, ix, iy): k for k, (l, ix, iy) in enumerate(np.asarray(leaves).tolist())}

    def find(l, I, J, mx, W, H):
        I %= (W * mx) << l
        J %= (H * mx) << l
        for l2 in (l, l - 1, l + 1):
            if l2 < 0:
                continue
            key = (l2, (I << max(0, l2 - l)) // mx >> max(0, l - l2), (J << max(0, l2 - l)) // mx >> max(0, l - l2))
            if key in d:
                return d[key], l2
        raise AssertionError("uncovered")
    return find


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oriented_brick_fill_equals_aligned(O, seed):
    """Ghost fill on a brick of mixed orientations, mapped back to brick
    directions, equals the aligned brick's fill: copies bit for bit; an
    averaged finer neighbour (and an interpolation whose coarse stencil
    reads one) within rounding of the four-term sum."""
    mx = 8
    L = S.random_balanced_leaves(seed, 1, 3, brick=BR)
    orient = codes(seed, BR)
    rng = np.random.default_rng(seed)
    q = rng.random((len(L), 1, mx, mx))
    kw = dict(mx=mx, velocity="constant", vel_params=(0.5, 0.3, 0.0), lmin=1, lmax=3)
    a = O.Oracle(L, brick=BR, **kw)
    a.set_interior(q)
    a.ghost_fill()
    b = oriented(O, L, BR, orient, **kw)
    b.set_interior(S.brick_own_data(q, L, BR, orient))
    b.ghost_fill()
    assert a.error == 0 and b.error == 0
    fa = a.full()
    fb = S.brick_aligned_data(b.full(), L, BR, orient, ghosts=2)
    assert not np.isnan(fb).any()
    diff = fa != fb
    find = _leaf_at(L)
    for k, f, j, i in zip(*np.nonzero(diff)):
        l, ix, iy = (int(v) for v in L[k])
        _, lc = find(l, ix * mx + i - 2, iy * mx + j - 2, mx, *BR)
        assert lc != l, "copied ghost cells are bit for bit"
        assert abs(fa[k, f, j, i] - fb[k, f, j, i]) <= 8 * np.spacing(1.0)
    assert diff.sum() < 0.5 * fa.size


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oriented_brick_steps_equal_aligned(O, seed):
    """Multirate coarse steps on a brick of mixed orientations equal the
    aligned brick's up to rounding order (the same discrete problem)."""
    mx = 8
    L = S.random_balanced_leaves(seed + 10, 1, 3, brick=BR)
    orient = codes(seed + 10, BR)
    q = S.sample_on_leaves(lambda x, y: 1.0 + np.exp(-20 * ((x - 1.2) ** 2 + (y - 0.9) ** 2)), L, mx)
    kw = dict(mx=mx, velocity="constant", vel_params=(0.5, -0.35, 0.0), lmin=1, lmax=3)
    a = O.Oracle(L, brick=BR, **kw)
    a.set_interior(q)
    b = oriented(O, L, BR, orient, **kw)
    b.set_interior(S.brick_own_data(q, L, BR, orient))
    dt = 0.8 / (mx << 1)
    for s in range(4):
        ca = a.coarse_step(s * dt, dt)
        cb = b.coarse_step(s * dt, dt)
        assert abs(ca - cb) <= 1e-15 * ca
    qa = a.interior()
    qb = S.brick_aligned_data(b.interior(), L, BR, orient)
    assert np.abs(qa - qb).max() < 1e-13
    # the data moved: a wrong transform could not hide behind a steady state
    assert np.abs(qa - q).max() > 1e-2


# ---------------------------------------------------------------------------
# mesh rules across block boundaries
# ---------------------------------------------------------------------------

def test_brick_mesh_rejections(O):
    """Tiling and 2:1 balance are checked in the brick's geometry: a missing
    block, and a level-3 leaf against a level-1 leaf across a block face, are
    rejected in every orientation of the finer block; the balanced mesh is
    accepted.  A brick takes only periodic constant-velocity advection."""
    L = S.uniform_leaves(1, (2, 1))
    with pytest.raises(O.OracleError):
        O.Oracle(L[L[:, 1] < 2], brick=(2, 1), lmin=1, lmax=3)      # block 1 missing
    # block 1's lower-left level-1 leaf refined twice at the face x = 1
    k = [tuple(v) for v in L.tolist()].index((1, 2, 0))
    R = S.refine_leaves(L, [k])
    k2 = [tuple(v) for v in R.tolist()].index((2, 4, 0))
    bad = S.refine_leaves(R, [k2])
    for code in range(8):
        orient = [0, code]
        with pytest.raises(O.OracleError):
            oriented(O, bad, (2, 1), orient, lmin=1, lmax=3)
        oriented(O, S.balance_leaves(bad, brick=(2, 1)), (2, 1), orient, lmin=1, lmax=3)
    for kw in (dict(equation="swe", velocity="none"), dict(velocity="swirl", vel_params=(1.0, 0, 0)),
               dict(bc=("reflect",) * 4)):
        with pytest.raises(O.OracleError):
            O.Oracle(L, brick=(2, 1), lmin=1, lmax=3, **kw)
    with pytest.raises(O.OracleError):
        O.Oracle(S.uniform_leaves(1), brick=(1, 1), orient=[8], lmin=1, lmax=3)


@pytest.mark.parametrize("smooth", [False, True])
def test_adapt_and_transfer_on_oriented_brick(O, smooth):
    """Adaptation (Sec. 4.1, smooth refinement of Sec. 4.2) decides in the
    brick's geometry: on a brick of mixed orientations it yields the aligned
    brick's leaf set (in own coordinates), and the transfer gives the aligned
    transfer's data in own indices (children interpolated bit for bit,
    parents averaged up to rounding order)."""
    mx = 8
    L = S.random_balanced_leaves(5, 1, 3, brick=BR)
    orient = codes(5, BR)
    rng = np.random.default_rng(5)
    q = rng.random((len(L), 1, mx, mx))
    tags = rng.choice([-1, 0, 1], size=len(L), p=[0.5, 0.3, 0.2]).astype(np.int8)
    kw = dict(mx=mx, velocity="constant", vel_params=(0.5, 0.3, 0.0), lmin=1, lmax=4)
    a = O.Oracle(L, brick=BR, **kw)
    a.set_interior(q)
    b = oriented(O, L, BR, orient, **kw)
    b.set_interior(S.brick_own_data(q, L, BR, orient))
    na = a.adapt(tags, smooth=smooth)
    nb = b.adapt(tags, smooth=smooth)
    assert sorted(map(tuple, S.brick_own_leaves(na, BR, orient).tolist())) == sorted(map(tuple, nb.tolist()))
    assert len(na) != len(L)
    a.ghost_fill()
    b.ghost_fill()
    a.regrid(na)
    b.regrid(S.brick_own_leaves(na, BR, orient))
    qa, qb = a.interior(), S.brick_aligned_data(b.interior(), na, BR, orient)
    assert np.abs(qa - qb).max() <= 4 * np.spacing(1.0)
