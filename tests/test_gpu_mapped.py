"""Mapped grids on the GPU (Sec. 1 metric terms; Sec. 5.2 runs a mapped
grid) against the oracle.

The computational square is mapped by X = (xi, eta) + alpha sin(2 pi xi)
sin(2 pi eta) (1, 1).  The GPU steps in capacity form with per-level tables
of the closed-form cell areas and averages fine cells by area in the ghost
fill and in coarsening; the oracle integrates the Jacobian over each cell by
Gauss-Legendre quadrature and scatters the transverse waves edge by edge (no
shared code).  Tolerance: the relative max-norm bar of the other parity
tests, 1e-12.  The coarsest level has at least 32 cells per axis, where the
oracle's quadrature is exact to rounding (its error term falls as h^8).
"""
import numpy as np
import pytest
import torch

from workloads import synth as S

pytestmark = pytest.mark.gpu
TOL = 1e-12
ALPHA = 0.1


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


def mapped_pair(B, O, L, mx, q, velocity="swirl", vel_params=(1.0, 0.0, 0.0), limiter="mc", lmin=None, lmax=None,
                alpha=ALPHA, capacity=None, time_stepping="multirate"):
    lv = np.asarray(L)
    lmin = int(lv[:, 0].min()) if lmin is None else lmin
    lmax = int(lv[:, 0].max()) if lmax is None else lmax
    ps = B.PatchStore(L, mx=mx, velocity=velocity, vel_params=vel_params, limiter=limiter, min_level=lmin,
                      max_level=lmax, capacity=capacity, map_alpha=alpha, time_stepping=time_stepping)
    ps.set_interior(q)
    o = O.Oracle(L, mx=mx, velocity=velocity, vel_params=vel_params, limiter=limiter, lmin=lmin, lmax=lmax,
                 map_alpha=alpha)
    o.set_interior(q)
    return ps, o


def hump(x, y):
    return 1.0 + np.exp(-30 * ((x - 0.45) ** 2 + (y - 0.55) ** 2))


# coarsest level 32 cells per axis or more
CASES = [(8, 2, 4), (16, 1, 3), (32, 0, 2)]


@pytest.mark.parametrize("mx,lmin,lmax", CASES)
@pytest.mark.parametrize("seed", range(2))
def test_mapped_fill_matches_oracle(B, O, mx, lmin, lmax, seed):
    """Ghost fill over all levels: copies, area-weighted eq. ghost_coarse
    averages (directly and inside the eq. ghost_fine stencils) against the
    oracle; the averages differ from the Cartesian ones."""
    if mx == 32 and lmin == 0:
        L = S.refine_leaves(S.refine_leaves(S.uniform_leaves(0), [0]), [0, 3])
    else:
        L = S.random_balanced_leaves(seed, lmin, lmax)
    q = np.random.default_rng(seed).random((len(L), 1, mx, mx))
    ps, o = mapped_pair(B, O, L, mx, q, lmin=lmin, lmax=lmax)
    ps.ghost_fill()
    o.ghost_fill()
    ps.check()
    ref = o.full()
    got = ps.patches().cpu().numpy()
    assert not np.isnan(ref).any()
    assert rel(got, ref) <= TOL
    flat, _ = mapped_pair(B, O, L, mx, q, lmin=lmin, lmax=lmax, alpha=0.0)
    flat.ghost_fill()
    assert rel(flat.patches(), ref) > 1e-6  # the weights matter


@pytest.mark.parametrize("limiter", ["mc", "lw", "minmod", "first"])
@pytest.mark.parametrize("mx,lmin,lmax", CASES)
def test_mapped_multirate_steps_match_oracle(B, O, limiter, mx, lmin, lmax):
    """Multirate coarse steps (Sec. 2.2) in capacity form through the swirl,
    every limiter, with the Courant number of the steps."""
    L = S.random_balanced_leaves(5, lmin, lmax) if lmin > 0 else \
        S.refine_leaves(S.refine_leaves(S.uniform_leaves(0), [0]), [0, 3])
    q = S.sample_on_leaves(hump, L, mx)
    ps, o = mapped_pair(B, O, L, mx, q, limiter=limiter, lmin=lmin, lmax=lmax)
    dt = 0.3 / (mx << lmin)
    n = 4
    c_o = 0.0
    for s in range(n):
        c_o = max(c_o, o.coarse_step(s * dt, dt))
    cfl = torch.zeros(1, dtype=torch.float64, device="cuda")
    ps.coarse_steps(dt, n, "per_level", cfl=cfl)
    ps.check()
    ref = o.interior()
    assert rel(ps.interior(), ref) <= TOL
    assert np.abs(ref - q).max() > 1e-2  # the data moved
    assert abs(cfl.item() - c_o) <= 1e-13 * c_o


@pytest.mark.parametrize("vel", [(0.7, -0.4), (-0.5, 0.9)])
def test_mapped_global_steps_constant_velocity(B, O, vel):
    """Global time stepping (every level at the finest step) at a constant
    velocity on a two-level mesh."""
    mx = 16
    L = S.random_balanced_leaves(3, 1, 3)
    q = S.sample_on_leaves(hump, L, mx)
    vp = (vel[0], vel[1], 0.0)
    ps, o = mapped_pair(B, O, L, mx, q, velocity="constant", vel_params=vp, time_stepping="global")
    dt = 0.3 / (mx << 3)
    for s in range(5):
        o.coarse_step(s * dt, dt, mode="global")
    ps.coarse_steps(dt, 5, "per_level")
    ps.check()
    assert rel(ps.interior(), o.interior()) <= TOL


def test_mapped_single_level_step_and_cfl(B, O):
    """One capacity-form step of a uniform level: values and Courant number
    (dt / (kappa h) of the cell a wave enters times its speed)."""
    mx, l = 16, 2
    L = S.uniform_leaves(l)
    q = np.random.default_rng(9).random((len(L), 1, mx, mx))
    ps, o = mapped_pair(B, O, L, mx, q)
    ps.ghost_fill()
    o.ghost_fill()
    dt = 0.4 / (mx << l)  # the smallest cells (kappa near 0.37) set the Courant number
    cfl = torch.zeros(1, dtype=torch.float64, device="cuda")
    ps.advance_level(l, 0.21, dt, cfl)
    c_o = o.advance_level(l, 0.21, dt)
    assert rel(ps.interior(), o.interior()) <= TOL
    assert abs(cfl.item() - c_o) <= 1e-13 * c_o
    # the capacity raises some cells' Courant numbers above the Cartesian one
    flat, fo = mapped_pair(B, O, L, mx, q, alpha=0.0)
    flat.ghost_fill()
    cf = torch.zeros(1, dtype=torch.float64, device="cuda")
    flat.advance_level(l, 0.21, dt, cf)
    assert cfl.item() > cf.item() * 2.0


def test_mapped_mass_conserved_on_uniform_level(B, O):
    """On a periodic uniform level the capacity form conserves the mass
    sum(kappa q) to rounding (the kappa from the oracle's quadrature)."""
    mx, l = 32, 1
    L = S.uniform_leaves(l)
    q = S.sample_on_leaves(hump, L, mx)
    ps, o = mapped_pair(B, O, L, mx, q)
    kap = np.zeros_like(q)
    for k, (lev, ix, iy) in enumerate(np.asarray(L).tolist()):
        for j in range(mx):
            for i in range(mx):
                kap[k, 0, j, i] = o.capacity(lev, ix * mx + i, iy * mx + j)
    m0 = float((kap * q).sum())
    ps.coarse_steps(0.35 / (mx << l), 12, "per_level")
    ps.check()
    m1 = float((kap * ps.interior().cpu().numpy()).sum())
    assert abs(m1 - m0) <= 1e-13 * abs(m0)


@pytest.mark.parametrize("smooth", [False, True])
def test_mapped_regrid_matches_oracle(B, O, smooth):
    """Tag, adapt, transfer (area-weighted coarsening) and the next coarse
    steps against the oracle; leaf sets exact."""
    mx = 16
    L = S.random_balanced_leaves(11, 1, 3)
    q = S.sample_on_leaves(lambda x, y: np.exp(-40 * ((x - 0.3) ** 2 + (y - 0.6) ** 2)), L, mx)
    ps, o = mapped_pair(B, O, L, mx, q, lmin=1, lmax=4, capacity=4 * len(L))
    ps.ghost_fill()
    o.ghost_fill()
    tags, _ = ps.tag(0.05, 0.02)
    otags, _ = o.tag(0.05, 0.02)
    tags = tags.cpu().numpy()
    assert np.array_equal(tags, otags)
    assert (tags < 0).any()  # some leaves coarsen
    new = ps.adapt(tags, smooth)
    assert np.array_equal(new, o.adapt(otags, smooth=smooth))
    ps.regrid(new)
    o.regrid(new)
    assert rel(ps.interior(), o.interior()) <= TOL
    dt = 0.3 / (mx << 1)
    for s in range(2):
        o.coarse_step(s * dt, dt)
    ps.coarse_steps(dt, 2, "per_level")
    ps.check()
    assert rel(ps.interior(), o.interior()) <= TOL


def test_mapped_coarsening_is_area_weighted(B, O):
    """Regrid that coarsens two sibling quartets and refines one leaf away
    from them: the new coarse cells are the area-weighted means of their
    children (mass kept), against the oracle."""
    mx = 16
    L = S.uniform_leaves(3)
    q = np.random.default_rng(4).random((len(L), 1, mx, mx))
    ps, o = mapped_pair(B, O, L, mx, q, lmin=2, lmax=4, capacity=128)
    kids = lambda ix, iy: {(3, 2 * ix + a, 2 * iy + b) for a in (0, 1) for b in (0, 1)}
    gone = kids(0, 0) | kids(1, 1) | {(3, 5, 5)}
    new = [[2, 0, 0], [2, 1, 1]] + [t for t in np.asarray(L).tolist() if tuple(t) not in gone]
    new += [[4, 10 + a, 10 + b] for b in (0, 1) for a in (0, 1)]
    new = np.asarray(new, dtype=np.int32)
    ps.regrid(new)
    o.regrid(new)
    ps.check()
    got = ps.interior().cpu().numpy()
    assert rel(got, o.interior()) <= TOL
    # coarse cell (0, 0) of the new leaf (2, 0, 0): its four children are
    # cells (0..1, 0..1) of the old leaf (3, 0, 0), weighted by their areas
    k0 = [tuple(t) for t in np.asarray(L).tolist()].index((3, 0, 0))
    y = q[k0, 0, :2, :2]
    a = np.array([[o.capacity(3, i, j) for i in range(2)] for j in range(2)])
    want = (a * y).sum() / a.sum()
    assert abs(got[0, 0, 0, 0] - want) <= 1e-13
    assert abs(y.mean() - want) > 1e-6


@pytest.mark.parametrize("mode", ["graph", "fused_levels", "fused", "persistent_graph"])
@pytest.mark.parametrize("mx,lmin,lmax", CASES)
def test_mapped_gathering_forms_match_per_level(B, O, mode, mx, lmin, lmax):
    """The ghost-gathering forms (a capacity-form kernel that gathers its
    ghosts, area-weighted averages included: one per level-step, launched from
    the host or replayed from a graph, or the persistent kernel walking the
    schedule) give the per-level form's bits, and the oracle's values, over
    multirate steps."""
    L = S.random_balanced_leaves(6, lmin, lmax) if lmin > 0 else \
        S.refine_leaves(S.refine_leaves(S.uniform_leaves(0), [0]), [0, 3])
    q = S.sample_on_leaves(hump, L, mx)
    a, o = mapped_pair(B, O, L, mx, q, lmin=lmin, lmax=lmax)
    b, _ = mapped_pair(B, O, L, mx, q, lmin=lmin, lmax=lmax)
    dt = 0.3 / (mx << lmin)
    n = 5
    ca = torch.zeros(1, dtype=torch.float64, device="cuda")
    cb = torch.zeros(1, dtype=torch.float64, device="cuda")
    a.coarse_steps(dt, n, "per_level", cfl=ca)
    b.coarse_steps(dt, n, mode, cfl=cb)
    a.check()
    b.check()
    assert np.array_equal(a.interior().cpu().numpy(), b.interior().cpu().numpy())
    assert ca.item() == cb.item()
    for s_ in range(n):
        o.coarse_step(s_ * dt, dt)
    assert rel(b.interior(), o.interior()) <= TOL


def test_mapped_store_rejects_other_forms(B, O):
    """The uniform-level step and the adjoint are Cartesian: they refuse a
    mapped store with FC_ERR_ARG, leaving the data untouched; the tuner picks
    one of the capacity-form kernel's own variants."""
    mx = 16
    L = S.uniform_leaves(1)
    q = np.random.default_rng(2).random((len(L), 1, mx, mx))
    ps, _ = mapped_pair(B, O, L, mx, q)
    qt = torch.as_tensor(q, device="cuda")
    with pytest.raises(B.FcError):
        ps.step_uniform(1, 0.0, 0.01, qt)
    with pytest.raises(B.FcError):
        ps.adjoint_step(1, 0.0, 0.01, qt, qt)
    assert ps.autotune() in (64, 128, 256)
    with pytest.raises(B.FcError):
        ps.set_variant(512)
    ps.check()
    assert np.array_equal(ps.interior().cpu().numpy(), q)


def test_full_size_mapped_mass_and_courant_l8(B):
    """At the benchmark's size (uniform level 8, 65536 patches of 32x32, the
    launch the mapped bench times): five steps keep the mass sum(kappa q) to
    rounding, with kappa the closed-form area factor
    1 + 2 pi alpha sigma^2 sin(2 pi (xi_c + eta_c)) (pinned against the
    oracle's quadrature), and the reported Courant number stays within the
    bound of the smallest cell, dt max|u| / (h (1 - 2 pi alpha sigma^2))."""
    mx, l = 32, 8
    w = S.workload("swirl_uniform", level=l, mx=mx, steps=5)
    dt = w["dt_coarse"] * (1.0 - 2.0 * np.pi * ALPHA)
    ps = B.PatchStore(w["leaves"], mx=mx, velocity="swirl", vel_params=w["vel_params"], min_level=l, max_level=l,
                      map_alpha=ALPHA)
    ps.set_interior(w["q0"])
    n = mx << l
    h = 1.0 / n
    sig = np.sin(np.pi * h) / (np.pi * h)
    lv = torch.as_tensor(np.asarray(w["leaves"]), device="cuda")
    ii = torch.arange(mx, device="cuda", dtype=torch.float64)
    I = lv[:, 1, None, None].double() * mx + ii[None, None, :]
    J = lv[:, 2, None, None].double() * mx + ii[None, :, None]
    kap = 1.0 + 2.0 * np.pi * ALPHA * sig * sig * torch.sin(2.0 * np.pi * (I + J + 1.0) * h)
    m0 = float((kap * ps.interior()[:, 0]).sum())
    cfl = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = 0.0
    for _ in range(5):
        ps.ghost_fill()
        ps.advance_level(l, t, dt, cfl)
        t += dt
    ps.check()
    q = ps.interior()[:, 0]
    m1 = float((kap * q).sum())
    assert abs(m1 - m0) <= 1e-12 * abs(m0)
    assert torch.isfinite(q).all()
    # swirl speeds are at most 1 (sin^2 sin products)
    assert 0.0 < cfl.item() <= dt / (h * (1.0 - 2.0 * np.pi * ALPHA * sig * sig)) * (1 + 1e-12)


@pytest.mark.parametrize("mx,nts", [(8, (64, 128)), (16, (64, 128, 256)), (32, (128, 256, 512))])
def test_mapped_launch_variants_bitwise_equal(B, O, mx, nts):
    """Every launch variant of the capacity-form kernel computes the same
    bits (each edge and cell is evaluated by the same expression)."""
    L = S.uniform_leaves(6 - {8: 0, 16: 1, 32: 2}[mx] - 2)
    q = np.random.default_rng(mx).random((len(L), 1, mx, mx))
    outs = []
    for nt in nts:
        ps, _ = mapped_pair(B, O, L, mx, q)
        ps.set_variant(nt)
        ps.coarse_steps(0.3 / (mx << int(np.asarray(L)[0, 0])), 3, "per_level")
        ps.check()
        outs.append(ps.interior().cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_mapped_adaptive_steps_with_rejection(B, O):
    """Clawpack-style adaptive coarse steps on the mapped grid (per-level
    form, cfl_max 1, target 0.9): the Courant number includes the cell areas,
    so the first try, sized for the Cartesian grid, is rejected; step sizes,
    accepted and rejected counts and the state against the same rule driven
    with the oracle."""
    from tests.test_gpu_contracts import oracle_adaptive
    mx = 16
    L = S.random_balanced_leaves(8, 1, 3)
    q = S.sample_on_leaves(hump, L, mx)
    ps = B.PatchStore(L, mx=mx, velocity="swirl", vel_params=(1.0, 0.0, 0.0), min_level=1, max_level=3,
                      map_alpha=ALPHA, cfl_max=1.0)
    ps.set_interior(q)
    o = O.Oracle(L, mx=mx, velocity="swirl", vel_params=(1.0, 0.0, 0.0), lmin=1, lmax=3, map_alpha=ALPHA)
    o.set_interior(q)
    dt0 = 0.9 / (mx << 1)  # Courant number 0.9 on the Cartesian grid
    t_end = 0.05
    dt_g, acc_g, rej_g = ps.advance_adaptive(t_end, dt0, 0.9, "per_level")
    t_o, dt_o, acc_o, rej_o = oracle_adaptive(o, t_end, dt0, 0.9, 1.0)
    ps.check()
    assert ps.time == t_end and t_o == t_end
    assert rej_g == rej_o >= 1 and acc_g == acc_o >= 3
    assert abs(dt_g - dt_o) <= 1e-12 * dt_o
    assert rel(ps.interior(), o.interior()) <= TOL
