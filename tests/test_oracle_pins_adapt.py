"""Pins of the oracle's adaptation with smooth refinement (Sec. 4.1, 4.2).

Sec. 4.2: every patch has a target level (its level, one more if tagged for
refinement, one less if tagged for coarsening); adaptation receives, for each
patch, the maximum target over the patch and all its neighbours; 2:1
balancing follows.  The checks below are properties that rule must have on
random meshes and tags, and one closed-form case: a refined patch gets a
buffer of refined neighbours, and a feature that stays put keeps the mesh
fixed.
"""
import numpy as np
import pytest

from workloads import synth as S


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def covered_levels(leaves, l, ix, iy):
    """Levels of the leaves inside or containing quadrant (l, ix, iy)."""
    out = []
    for (L, x, y) in leaves:
        if L >= l:
            if (x >> (L - l)) == ix and (y >> (L - l)) == iy:
                out.append(L)
        elif (ix >> (l - L)) == x and (iy >> (l - L)) == y:
            out.append(L)
    return out


def neighbours(leaves, k, periodic=True):
    """Indices of the leaves touching leaf k across a face or a corner."""
    l, ix, iy = leaves[k]
    res = set()
    for j, (L, x, y) in enumerate(leaves):
        if j == k:
            continue
        # both as intervals on the finest of the two levels, periodic distance
        m = max(l, L)
        n = 1 << m
        a0, a1 = ix << (m - l), (ix + 1) << (m - l)
        b0, b1 = x << (m - L), (x + 1) << (m - L)
        c0, c1 = iy << (m - l), (iy + 1) << (m - l)
        d0, d1 = y << (m - L), (y + 1) << (m - L)

        def touch(p0, p1, q0, q1):
            for sh in ((-n, 0, n) if periodic else (0,)):
                if q0 + sh <= p1 and p0 <= q1 + sh:
                    return True
            return False
        if touch(a0, a1, b0, b1) and touch(c0, c1, d0, d1):
            res.add(j)
    return res


def random_case(seed, lmin=2, lmax=5):
    L = S.random_balanced_leaves(seed, lmin, 4)
    rng = np.random.default_rng(seed)
    tags = rng.choice([-1, 0, 0, 1], size=len(L), p=[0.5, 0.15, 0.15, 0.2]).astype(np.int8)
    return [tuple(x) for x in L.tolist()], tags, lmin, lmax


@pytest.mark.parametrize("seed", range(6))
def test_smooth_adapt_properties(O, seed):
    """On random 2:1 meshes with random tags: the result tiles the square
    and is 2:1 balanced (the oracle accepts it); every leaf tagged for
    refinement is refined; every neighbour of such a leaf P (level l) ends,
    over its whole area, at least one level finer if it was not finer than
    P, or not coarser than it was; every new parent comes from four leaves
    whose own targets and all of whose neighbours' targets were below the
    children's level."""
    leaves, tags, lmin, lmax = random_case(seed)
    o = O.Oracle(leaves, mx=8, lmin=lmin, lmax=lmax)
    new = [tuple(x) for x in o.adapt(tags, smooth=True).tolist()]
    O.Oracle(new, mx=8, lmin=lmin, lmax=lmax)              # raises unless balanced and tiling
    newset = set(new)
    target = [min(lmax, max(lmin, l + int(t))) for (l, _, _), t in zip(leaves, tags)]
    for k, (l, ix, iy) in enumerate(leaves):
        if tags[k] == 1 and l < lmax:
            assert (l, ix, iy) not in newset
            for j in neighbours(leaves, k):
                lj = leaves[j][0]
                want = min(lj + 1, lmax) if lj <= l else lj
                assert min(covered_levels(new, *leaves[j])) >= want, (leaves[k], leaves[j])
    old = {x: k for k, x in enumerate(leaves)}
    for (l, ix, iy) in new:
        kids = [(l + 1, 2 * ix + cx, 2 * iy + cy) for cy in (0, 1) for cx in (0, 1)]
        if all(c in old for c in kids):
            for c in kids:
                kc = old[c]
                assert target[kc] < l + 1
                for j in neighbours(leaves, kc):
                    assert target[j] < l + 1


def test_smooth_refinement_buffer_and_fixed_feature(O):
    """One tagged patch in a uniform level-2 mesh: it and its eight
    neighbours are refined (a buffer of refined patches around it, the
    'additional layer' of Sec. 4.2), nothing else.  Re-tagging with the
    feature in the same place (the four children of the tagged patch kept,
    every other level-3 patch tagged for coarsening) leaves the mesh as it
    is: each coarsening family touches a kept child."""
    L = [tuple(x) for x in S.uniform_leaves(2).tolist()]
    o = O.Oracle(L, mx=8, lmin=2, lmax=3)
    k0 = L.index((2, 1, 2))
    tags = np.zeros(len(L), dtype=np.int8)
    tags[k0] = 1
    new = [tuple(x) for x in o.adapt(tags, smooth=True).tolist()]
    refined = {(ix, iy) for (l, ix, iy) in L if (l + 1, 2 * ix, 2 * iy) in set(new)}
    assert refined == {(x % 4, y % 4) for x in (0, 1, 2) for y in (1, 2, 3)}
    assert len(new) == 16 - 9 + 36
    # without smoothing only the tagged patch refines (plus nothing: the mesh stays 2:1)
    plain = [tuple(x) for x in o.adapt(tags, smooth=False).tolist()]
    assert len(plain) == 16 - 1 + 4
    # the feature stays: children of the tagged patch kept, the rest of level 3 coarsen
    o2 = O.Oracle(new, mx=8, lmin=2, lmax=3)
    feat = {(3, 2 * 1 + cx, 2 * 2 + cy) for cx in (0, 1) for cy in (0, 1)}
    tags2 = np.array([0 if (x in feat or x[0] == 2) else -1 for x in new], dtype=np.int8)
    again = [tuple(x) for x in o2.adapt(tags2, smooth=True).tolist()]
    assert sorted(again) == sorted(new)
    # without smoothing the buffer would coarsen away
    assert len(o2.adapt(tags2, smooth=False)) < len(new)


def test_smooth_equals_plain_when_neighbours_agree(O):
    """All tags equal: every neighbour's target is the leaf's own level plus
    the same tag on a uniform mesh, so the maximum changes nothing."""
    L = S.uniform_leaves(3)
    o = O.Oracle(L, mx=8, lmin=2, lmax=4)
    for t in (-1, 0, 1):
        tags = np.full(len(L), t, dtype=np.int8)
        assert np.array_equal(o.adapt(tags, smooth=True), o.adapt(tags, smooth=False))
