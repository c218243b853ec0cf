"""Multiblock brick on the GPU (Sec. 2.3 index transforms) against the oracle.

Every neighbour record of a brick store carries the index transform between
the two patches (eq. transform: a signed permutation A and a translation F);
the gather kernels apply it to copies, eq. ghost_coarse averages and eq.
ghost_fine interpolations, and each patch advances in its block's own index
directions.  These tests run bricks of mixed orientations through the C ABI
and compare with the oracle, which carries indices through the brick's
coordinates by point location instead (no shared code).  Tolerance: the
relative max-norm bar of the other parity tests, 1e-12; the replicated
layout and the Courant-one shift are compared bit for bit (GPU against GPU,
and against the exact shift).
"""
import numpy as np
import pytest
import torch

from workloads import synth as S

pytestmark = pytest.mark.gpu
TOL = 1e-12
BR = (3, 2)
ALL8 = (4, 2)


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1703_03116_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def rel(a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def brick_pair(B, O, leaves_brick, brick, orient, mx, q_brick, vel=(0.5, 0.3), lmin=None, lmax=None,
               limiter="mc", capacity=None):
    """GPU store and oracle on the same oriented brick; leaves and data given
    in brick coordinates and directions, handed over in own ones."""
    own = S.brick_own_leaves(leaves_brick, brick, orient)
    q = S.brick_own_data(q_brick, leaves_brick, brick, orient)
    lv = np.asarray(leaves_brick)
    lmin = int(lv[:, 0].min()) if lmin is None else lmin
    lmax = int(lv[:, 0].max()) if lmax is None else lmax
    vp = (vel[0], vel[1], 0.0)
    ps = B.PatchStore(own, mx=mx, velocity="constant", vel_params=vp, limiter=limiter, min_level=lmin,
                      max_level=lmax, capacity=capacity, brick=brick, orient=orient)
    ps.set_interior(q)
    o = O.Oracle(own, mx=mx, velocity="constant", vel_params=vp, limiter=limiter, lmin=lmin, lmax=lmax,
                 brick=brick, orient=orient)
    o.set_interior(q)
    return ps, o


def orient_of(seed, brick):
    return [int(v) for v in np.random.default_rng(100 + seed).integers(0, 8, brick[0] * brick[1])]


@pytest.mark.parametrize("mx", [8, 16, 32])
@pytest.mark.parametrize("seed", range(3))
def test_brick_fill_matches_oracle(B, O, mx, seed):
    """Ghost fill over all levels of a mixed-orientation brick: every ghost
    cell (copies, averages, interpolations across rotated and reflected block
    faces and corners) against the oracle."""
    L = S.random_balanced_leaves(seed, 1, 3, brick=BR)
    orient = orient_of(seed, BR)
    q = np.random.default_rng(seed).random((len(L), 1, mx, mx))
    ps, o = brick_pair(B, O, L, BR, orient, mx, q)
    ps.ghost_fill()
    o.ghost_fill()
    ps.check()
    ref = o.full()
    assert not np.isnan(ref).any()
    got = ps.patches().cpu().numpy()
    assert rel(got, ref) <= TOL
    # copies are exact: most ghost cells agree bit for bit
    assert (got == ref).mean() > 0.9


@pytest.mark.parametrize("mode", ["per_level", "graph", "fused_levels", "fused", "persistent_graph"])
@pytest.mark.parametrize("mx", [8, 16, 32])
def test_brick_multirate_steps_match_oracle(B, O, mode, mx):
    """Multirate coarse steps (Sec. 2.2 fill + advance per level-step) on a
    mixed-orientation brick, in every execution form, against the oracle."""
    seed = mx
    L = S.random_balanced_leaves(seed, 1, 3, brick=BR)
    orient = orient_of(seed, BR)
    q = S.sample_on_leaves(lambda x, y: 1.0 + np.exp(-8 * ((x - 1.3) ** 2 + (y - 0.8) ** 2)), L, mx)
    ps, o = brick_pair(B, O, L, BR, orient, mx, q, vel=(0.5, -0.35))
    dt = 0.8 / (mx << 1)
    n = 6
    for s in range(n):
        o.coarse_step(s * dt, dt)
    ps.coarse_steps(dt, n, mode)
    ps.check()
    ref = o.interior()
    assert rel(ps.interior(), ref) <= TOL
    assert np.abs(ref - q).max() > 1e-2  # the data moved


@pytest.mark.parametrize("vel", [(1.0, 1.0), (-1.0, 1.0)])
def test_brick_unit_courant_shift_all_orientations(B, vel):
    """At Courant number one the scheme shifts data one cell diagonally per
    step; on a brick of all eight orientations the GPU gives the exact shift
    in brick directions."""
    mx, l = 16, 1
    L = S.uniform_leaves(l, ALL8)
    orient = list(range(8))
    G0 = np.random.default_rng(3).random((ALL8[1] * mx << l, ALL8[0] * mx << l))
    qb = np.stack([[G0[iy * mx:(iy + 1) * mx, ix * mx:(ix + 1) * mx]] for (_, ix, iy) in L.tolist()])
    own = S.brick_own_leaves(L, ALL8, orient)
    ps = B.PatchStore(own, mx=mx, velocity="constant", vel_params=(vel[0], vel[1], 0.0), min_level=l,
                      max_level=l, brick=ALL8, orient=orient)
    ps.set_interior(S.brick_own_data(qb, L, ALL8, orient))
    h = 1.0 / (mx << l)
    ps.coarse_steps(h, 3, "graph")
    ps.check()
    got = S.brick_aligned_data(ps.interior().cpu().numpy(), L, ALL8, orient)
    G = np.zeros_like(G0)
    for (_, ix, iy), p in zip(L.tolist(), got):
        G[iy * mx:(iy + 1) * mx, ix * mx:(ix + 1) * mx] = p[0]
    ref = np.roll(np.roll(G0, 3 * int(vel[1]), 0), 3 * int(vel[0]), 1)
    assert np.abs(G - ref).max() < 1e-15


def test_replicated_aligned_brick_equals_one_block_bitwise(B):
    """The paper's replicated weak-scaling layout (Sec. 5.1): the same mesh
    and data in each block of an aligned periodic brick at u = (0.5, 0.5)
    give the one-block result in every block, bit for bit."""
    mx = 16
    one = S.random_balanced_leaves(4, 2, 4)
    q = np.random.default_rng(4).random((len(one), 1, mx, mx))
    kw = dict(mx=mx, velocity="constant", vel_params=(0.5, 0.5, 0.0), min_level=2, max_level=4)
    a = B.PatchStore(one, **kw)
    a.set_interior(q)
    nb = BR[0] * BR[1]
    b = B.PatchStore(S.replicate_leaves(one, BR), brick=BR, **kw)
    b.set_interior(np.concatenate([q] * nb))
    dt = 0.8 / (mx << 2)
    a.coarse_steps(dt, 5, "graph")
    b.coarse_steps(dt, 5, "graph")
    a.check()
    b.check()
    qa = a.interior().cpu().numpy()
    assert np.array_equal(b.interior().cpu().numpy(), np.concatenate([qa] * nb))


@pytest.mark.parametrize("smooth", [False, True])
def test_brick_regrid_matches_oracle(B, O, smooth):
    """Tag, adapt (host, in the brick's geometry) and transfer on a
    mixed-orientation brick: leaf sets exact, transferred data and the next
    coarse steps against the oracle."""
    mx = 16
    L = S.random_balanced_leaves(7, 1, 3, brick=BR)
    orient = orient_of(7, BR)
    q = S.sample_on_leaves(lambda x, y: np.exp(-6 * ((x - 1.6) ** 2 + (y - 1.1) ** 2)), L, mx)
    ps, o = brick_pair(B, O, L, BR, orient, mx, q, lmin=1, lmax=4, capacity=4 * len(L))
    ps.ghost_fill()
    o.ghost_fill()
    tags, _ = ps.tag(0.05, 0.02)
    otags, _ = o.tag(0.05, 0.02)
    tags = tags.cpu().numpy()
    assert np.array_equal(tags, otags)
    new = ps.adapt(tags, smooth)
    assert np.array_equal(new, o.adapt(otags, smooth=smooth))
    ps.regrid(new)
    o.regrid(new)
    assert rel(ps.interior(), o.interior()) <= TOL
    dt = 0.8 / (mx << 2)
    for s in range(2):
        o.coarse_step(s * dt, dt)
    ps.coarse_steps(dt, 2, "graph")
    ps.check()
    assert rel(ps.interior(), o.interior()) <= TOL
