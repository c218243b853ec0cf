"""GPU path (through the C ABI) against the FP64 CPU oracle.

Tolerance: relative max-norm ||gpu - oracle||_inf / ||oracle||_inf <= 1e-12
in FP64 for every floating-point result (the bar the target states);
integer results (tags, leaf sets) must match exactly.  Ghost copies are
compared bitwise.  Inputs are seeded and synthetic (workloads.synth).
"""
import numpy as np
import pytest
import torch

from workloads import synth as S

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def B():
    import torch
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


def pair(B, O, leaves, mx, q, equation="advection", velocity="constant", vel_params=(1.0, 0.5, 0.0),
         bc=("periodic",) * 4, lmin=None, lmax=None, limiter="mc", time_stepping="multirate", capacity=None):
    lv = np.asarray(leaves)
    lmin = int(lv[:, 0].min()) if lmin is None else lmin
    lmax = int(lv[:, 0].max()) if lmax is None else lmax
    ps = B.PatchStore(leaves, mx=mx, equation=equation, limiter=limiter, bc=bc, velocity=velocity,
                      vel_params=vel_params, min_level=lmin, max_level=lmax, time_stepping=time_stepping,
                      capacity=capacity)
    ps.set_interior(q)
    o = O.Oracle(leaves, mx=mx, equation=equation, limiter=limiter, bc=bc, velocity=velocity,
                 vel_params=vel_params, lmin=lmin, lmax=lmax)
    o.set_interior(q)
    return ps, o


def ghost_mask(mx, m=2):
    N = mx + 2 * m
    g = np.ones((N, N), dtype=bool)
    g[m:m + mx, m:m + mx] = False
    return g


# ---------------------------------------------------------------------------
# ghost filling
# ---------------------------------------------------------------------------

def test_fill_uniform_copy_bitwise(B, O):
    L = S.uniform_leaves(2)
    rng = np.random.default_rng(0)
    q = rng.random((16, 1, 8, 8))
    ps, o = pair(B, O, L, 8, q)
    ps.ghost_fill()
    o.ghost_fill()
    assert np.array_equal(ps.patches().cpu().numpy(), o.full())


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("bc", ["periodic", "reflect"])
def test_fill_amr_matches_algorithm1(B, O, seed, bc):
    per = bc == "periodic"
    L = S.random_balanced_leaves(seed, 2, 5 if seed % 2 else 4, periodic=(per, per))
    rng = np.random.default_rng(seed)
    eq = "advection" if per else "swe"
    F = 1 if per else 3
    q = 1.0 + rng.random((len(L), F, 8, 8))
    ps, o = pair(B, O, L, 8, q, equation=eq, velocity="constant" if per else "none", bc=(bc,) * 4)
    ps.ghost_fill()
    o.ghost_fill()
    ps.check()
    g, r = ps.patches().cpu().numpy(), o.full()
    assert not np.isnan(g).any()
    assert rel(g, r) <= 1e-14


def test_fill_time_interpolated_coarse_level(B, O):
    """Level l filled at half the coarse step: coarse data q_old + 1/2 (q - q_old)."""
    L = S.random_balanced_leaves(11, 2, 4)
    assert (np.asarray(L)[:, 0] == 4).sum() > 0
    rng = np.random.default_rng(11)
    q = rng.random((len(L), 1, 8, 8))
    ps, o = pair(B, O, L, 8, q, velocity="constant", vel_params=(0.7, -0.4, 0), lmin=2, lmax=4)
    for lo in (2, 3):
        ps.ghost_fill(lo, lo, 1.0)
        o.ghost_fill(lo, lo, 1.0)
        ps.advance_level(lo, 0.0, 0.01)
        o.advance_level(lo, 0.0, 0.01)
    for alpha in (0.0, 0.5):
        ps.ghost_fill(4, 4, alpha)
        o.ghost_fill(4, 4, alpha)
        lv = np.asarray(L)[:, 0]
        g, r = ps.patches().cpu().numpy()[lv == 4], o.full()[lv == 4]
        assert rel(g, r) <= 1e-14


# ---------------------------------------------------------------------------
# advance and multirate stepping
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("limiter", ["mc", "lw", "minmod"])
def test_single_step_uniform(B, O, limiter):
    L = S.uniform_leaves(2)
    rng = np.random.default_rng(1)
    q = rng.random((16, 1, 16, 16))
    ps, o = pair(B, O, L, 16, q, velocity="swirl", vel_params=(1.0, 0, 0), limiter=limiter)
    ps.ghost_fill()
    o.ghost_fill()
    cfl = __import__("torch").zeros(1, dtype=__import__("torch").float64, device="cuda")
    ps.advance_level(2, 0.13, 0.9 / 64, cfl)
    c_o = o.advance_level(2, 0.13, 0.9 / 64)
    assert rel(ps.interior(), o.interior()) <= TOL
    assert abs(cfl.item() - c_o) <= 1e-14


@pytest.mark.parametrize("mode", ["per_level", "fused", "graph", "fused_levels", "persistent_graph"])
def test_swirl_uniform_parity(B, O, mode):
    w = S.workload("swirl_uniform", level=3, mx=16)
    ps, o = pair(B, O, w["leaves"], 16, w["q0"], velocity="swirl", vel_params=(1.0, 0, 0))
    dt = w["dt_coarse"]
    ps.coarse_steps(dt, 40, mode)
    for s in range(40):
        o.coarse_step(s * dt, dt)
    ps.check()
    assert rel(ps.interior(), o.interior()) <= TOL


@pytest.mark.parametrize("mode", ["per_level", "fused", "graph", "fused_levels", "persistent_graph"])
def test_hump_multirate_parity(B, O, mode):
    """Levels 2-3 with subcycling, 8x8 patches, 100 coarse steps."""
    w = S.workload("hump_l23")
    ps, o = pair(B, O, w["leaves"], 8, w["q0"], velocity="constant", vel_params=w["vel_params"])
    dt = w["dt_coarse"]
    ps.coarse_steps(dt, w["steps"], mode)
    for s in range(w["steps"]):
        o.coarse_step(s * dt, dt)
    ps.check()
    assert rel(ps.interior(), o.interior()) <= TOL


@pytest.mark.parametrize("seed", [3, 4])
def test_random_amr_multirate_swirl(B, O, seed):
    """Random 2:1 meshes over levels 2-5 (ragged level populations)."""
    L = S.random_balanced_leaves(seed, 2, 5)
    q = S.sample_on_leaves(S.gaussians(S.gaussian_params(seed)), L, 8)
    ps, o = pair(B, O, L, 8, q, velocity="swirl", vel_params=(1.0, 0, 0))
    dt = 0.9 / 32
    for mode in ("fused", "per_level", "graph", "fused_levels"):
        ps.coarse_steps(dt, 3, mode)
    for s in range(12):
        o.coarse_step(s * dt, dt)
    ps.check()
    assert rel(ps.interior(), o.interior()) <= TOL


def test_global_stepping_parity(B, O):
    L = S.random_balanced_leaves(6, 2, 4)
    q = S.sample_on_leaves(S.gaussians(S.gaussian_params(6)), L, 8)
    ps, o = pair(B, O, L, 8, q, velocity="swirl", vel_params=(1.0, 0, 0), time_stepping="global")
    dt = 0.9 / 128
    ps.coarse_steps(dt, 5, "per_level")
    ps.coarse_steps(dt, 5, "graph")
    for s in range(10):
        o.coarse_step(s * dt, dt, "global")
    assert rel(ps.interior(), o.interior()) <= TOL


def test_fused_equals_per_level_bitwise(B, O):
    w = S.workload("hump_l23")
    a = B.from_workload(w)
    b = B.from_workload(w)
    a.coarse_steps(w["dt_coarse"], 20, "per_level")
    b.coarse_steps(w["dt_coarse"], 20, "graph")
    assert np.array_equal(a.interior().cpu().numpy(), b.interior().cpu().numpy())
    c = B.from_workload(w)
    c.coarse_steps(w["dt_coarse"], 7, "persistent_graph")
    c.coarse_steps(w["dt_coarse"], 13, "fused")
    assert np.array_equal(a.interior().cpu().numpy(), c.interior().cpu().numpy())


@pytest.mark.parametrize("mx", [8, 32])
def test_complete_level_fused_equals_per_level_bitwise(B, mx):
    """On a complete periodic level the fused kernels derive neighbour slots
    from the Morton index instead of reading records; the result must be
    the fill-then-advance result bit for bit."""
    w = S.workload("swirl_uniform", level=3 if mx == 8 else 2, mx=mx)
    a = B.from_workload(w)
    b = B.from_workload(w)
    a.coarse_steps(w["dt_coarse"], 6, "per_level")
    b.coarse_steps(w["dt_coarse"], 3, "graph")
    b.coarse_steps(w["dt_coarse"], 3, "fused_levels")
    assert np.array_equal(a.interior().cpu().numpy(), b.interior().cpu().numpy())


def test_graph_replays_track_parity_and_step(B):
    """Graph nodes carry the buffer parities and the coarse step as constants:
    replays from either parity, chunk and single-step graphs, and a change of
    step (recapture) must reproduce the host-driven sequence bit for bit,
    CFL numbers included."""
    w = S.workload("hump_l23")
    dt = w["dt_coarse"]
    plan = [(1, dt), (1, dt), (3, dt), (50, dt), (1, dt), (55, 0.5 * dt), (2, dt), (51, dt)]
    a = B.from_workload(w)
    b = B.from_workload(w)
    for n, h in plan:
        ca = torch.zeros(1, dtype=torch.float64, device="cuda")
        cb = torch.zeros(1, dtype=torch.float64, device="cuda")
        a.coarse_steps(h, n, "per_level", cfl=ca)
        b.coarse_steps(h, n, "graph", cfl=cb)
        assert np.array_equal(a.interior().cpu().numpy(), b.interior().cpu().numpy())
        assert float(ca) == float(cb) and float(ca) > 0.0
        assert a.time == b.time
    b.check()


@pytest.mark.parametrize("mode", ["graph", "persistent_graph"])
def test_prepared_graphs_replay_the_same_steps(B, mode):
    """Graphs captured ahead by prepare_steps (after an odd number of steps,
    so from the other parity) give the same bits as the on-demand ones, and
    prepare_steps itself changes neither the solution nor the time."""
    w = S.workload("hump_l23")
    dt = w["dt_coarse"]
    a = B.from_workload(w)
    b = B.from_workload(w)
    for ps in (a, b):
        ps.coarse_steps(dt, 3, "per_level")
    q3, t3 = b.interior().clone(), b.time
    b.prepare_steps(dt, 53, mode)
    assert torch.equal(b.interior(), q3) and b.time == t3
    a.coarse_steps(dt, 53, "per_level")
    b.coarse_steps(dt, 53, mode)
    assert torch.equal(a.interior(), b.interior())
    b.check()


def test_forms_bitwise_at_level_6(B):
    """4096 patches (85 MB of solution: the advance writes with plain
    stores at this size, with streaming stores below and above it): the
    graph form, the host-launched fused kernels and the per-level form take
    the same steps bit for bit, CFL numbers included."""
    w = S.workload("swirl_uniform", level=6, mx=32)
    dt = w["dt_coarse"]
    out, cfls = [], []
    for mode in ("graph", "fused_levels", "per_level"):
        ps = B.from_workload(w)
        cfl = torch.zeros(1, dtype=torch.float64, device="cuda")
        ps.coarse_steps(dt, 6, mode, cfl=cfl)
        ps.check()
        out.append(ps.interior())
        cfls.append(float(cfl))
    assert torch.equal(out[0], out[1]) and torch.equal(out[0], out[2])
    assert cfls[0] == cfls[1] == cfls[2] > 0.0


@pytest.mark.parametrize("mx", [8, 16, 32])
def test_variants_bitwise(B, mx):
    """Every launch variant (threads per patch x tile shape, i.e. cells per
    sweep segment) computes the same bits."""
    level = {8: 3, 16: 2, 32: 2}[mx]
    w = S.workload("swirl_uniform", level=level, mx=mx)
    nts = {8: [64, 128], 16: [64, 128, 256], 32: [128, 256, 512]}[mx]
    longs = {(16, 128): 8, (16, 256): 8, (32, 256): 16, (32, 512): 8}
    res, seen = [], []
    for nt in nts:
        for seg in (0, longs.get((mx, nt))):
            if seg is None:
                continue
            ps = B.from_workload(w)
            ps.set_variant(nt)
            ps.set_tile(seg)
            seen.append(ps.launch())
            ps.coarse_steps(w["dt_coarse"], 5, "fused")
            ps.coarse_steps(w["dt_coarse"], 5, "per_level")
            ps.coarse_steps(w["dt_coarse"], 5, "graph")
            res.append(ps.interior().cpu().numpy())
    assert len(set(seen)) == len(seen)
    for r in res[1:]:
        assert np.array_equal(r, res[0])


def test_replicated_blocks_identical(B):
    """Replicated initial data on a periodic uniform mesh: a field that
    repeats with period 1/2 stays periodic, bitwise, in every block."""
    L = S.uniform_leaves(3)
    q = S.sample_on_leaves(lambda x, y: np.exp(-((np.mod(x, 0.5) - 0.2) ** 2 + (np.mod(y, 0.5) - 0.3) ** 2) / 0.005),
                           L, 16)
    ps = B.PatchStore(L, mx=16, velocity="constant", vel_params=(0.6, -0.3, 0))
    ps.set_interior(q)
    ps.coarse_steps(0.9 / 128 / 0.6, 30, "graph")
    G = np.zeros((128, 128))
    qi = ps.interior().cpu().numpy()
    for k, (l, ix, iy) in enumerate(L):
        G[iy * 16:(iy + 1) * 16, ix * 16:(ix + 1) * 16] = qi[k, 0]
    for by in range(2):
        for bx in range(2):
            assert np.array_equal(G[by * 64:(by + 1) * 64, bx * 64:(bx + 1) * 64], G[:64, :64])


# ---------------------------------------------------------------------------
# tagging and regrid
# ---------------------------------------------------------------------------

def test_tag_and_adapt_parity(B, O):
    L = S.random_balanced_leaves(9, 2, 4)
    q = S.sample_on_leaves(S.gaussians(S.gaussian_params(9)), L, 8)
    ps, o = pair(B, O, L, 8, q, velocity="swirl", vel_params=(1.0, 0, 0), lmin=2, lmax=5, capacity=4 ** 5)
    ps.ghost_fill()
    o.ghost_fill()
    tg, g2 = ps.tag(2.0, 0.5)
    to, g2o = o.tag(2.0, 0.5)
    assert rel(g2, g2o) <= 1e-13
    assert np.array_equal(tg.cpu().numpy(), to)
    new_g = ps.adapt(tg)
    new_o = o.adapt(to)
    assert np.array_equal(new_g, new_o)
    ps.regrid(new_g)
    o.regrid(new_o)
    assert rel(ps.interior(), o.interior()) <= 1e-14
    dt = 0.9 / 32
    ps.coarse_steps(dt, 2, "graph")
    for s in range(2):
        o.coarse_step(s * dt, dt)
    assert rel(ps.interior(), o.interior()) <= TOL


# ---------------------------------------------------------------------------
# full size of the benchmark workload
# ---------------------------------------------------------------------------

def test_full_size_uniform_level5_swirl(B, O):
    """1024 patches of 32x32 (1024^2 cells), 500 steps, the benchmark's
    launch configuration (persistent kernel replayed from a graph)."""
    O.set_threads(max(1, min(16, O.max_threads())))
    w = S.workload("swirl_uniform", level=5, mx=32)
    ps = B.from_workload(w)
    ps.autotune()
    dt = w["dt_coarse"]
    ps.coarse_steps(dt, w["steps"], "graph")
    o = O.from_workload(w)
    for s in range(w["steps"]):
        o.coarse_step(s * dt, dt)
    ps.check()
    g = ps.interior().cpu().numpy()
    assert rel(g, o.interior()) <= TOL
    m0 = w["q0"].sum()
    assert abs(g.sum() - m0) / m0 < 1e-12


# ---------------------------------------------------------------------------
# shallow water (3-field SoA store, reflecting walls, Roe + entropy fix)
# ---------------------------------------------------------------------------

def swe_pair(B, O, w, mx):
    return pair(B, O, w["leaves"], mx, w["q0"], equation="swe", velocity="none", bc=("reflect",) * 4,
                lmin=w["lmin"], lmax=w["lmax"])


@pytest.mark.parametrize("mode", ["per_level", "fused", "graph"])
@pytest.mark.parametrize("mx", [8, 16])
def test_swe_dam_break_amr_parity(B, O, mode, mx):
    """Radial dam break on levels 2-4 with subcycling, fixed coarse step
    (Courant number <= 0.6 on the finest level for |u| + c <= 1.6)."""
    w = S.workload("dam_break", lmin=2, lmax=4, mx=mx)
    ps, o = swe_pair(B, O, w, mx)
    dt = 0.6 / (mx * 4) / 1.6
    ps.coarse_steps(dt, 6, mode)
    for s in range(6):
        o.coarse_step(s * dt, dt)
    ps.check()
    assert rel(ps.interior(), o.interior()) <= TOL


@pytest.mark.parametrize("mx,nts", [(16, (256, 384, 512, 640)), (8, (64, 128, 192))])
def test_swe_variants_bitwise(B, mx, nts):
    """Every shallow-water launch variant computes the same bits, in the
    graph form: each edge's update is the same code whichever thread runs
    it, and every per-cell accumulator receives exactly two contributions
    (one per edge of the cell) added to -0, so their order does not matter."""
    w = S.workload("dam_break", lmin=2, lmax=4, mx=mx)
    dt = 0.6 / (mx * 4) / 1.6
    res = []
    for nt in nts:
        ps = B.from_workload(w)
        ps.set_variant(nt)
        ps.coarse_steps(dt, 4, "graph")
        ps.check()
        res.append(ps.interior().cpu().numpy())
    for r in res[1:]:
        assert np.array_equal(r, res[0])


def test_swe_lake_at_rest_bitwise(B):
    L = S.random_balanced_leaves(3, 2, 4, periodic=(False, False))
    q = np.zeros((len(L), 3, 16, 16))
    q[:, 0] = 1.3
    ps = B.PatchStore(L, mx=16, equation="swe", velocity="none", bc=("reflect",) * 4)
    ps.set_interior(q)
    ps.coarse_steps(0.004, 4, "graph")
    assert np.array_equal(ps.interior().cpu().numpy(), q)


def test_swe_single_step_cfl(B, O):
    w = S.workload("dam_break", lmin=3, lmax=3, mx=16)
    ps, o = swe_pair(B, O, w, 16)
    import torch
    cfl = torch.zeros(1, dtype=torch.float64, device="cuda")
    ps.ghost_fill()
    o.ghost_fill()
    ps.advance_level(3, 0.0, 0.002, cfl)
    c_o = o.advance_level(3, 0.0, 0.002)
    assert rel(ps.interior(), o.interior()) <= TOL
    assert abs(cfl.item() - c_o) <= 1e-14 * c_o


def _oracle_run_adaptive(o, dt, ncoarse, regrid_every, tau_r, tau_c):
    t = 0.0
    for k in range(ncoarse):
        if k % regrid_every == 0 and k > 0:
            o.ghost_fill()
            tags, _ = o.tag(tau_r, tau_c)
            o.regrid(o.adapt(tags))
        o.coarse_step(t, dt)
        t = t + dt
    return t


@pytest.mark.parametrize("mx", [8, 16])
def test_adaptive_swirl_with_regrid(B, O, mx):
    """Levels 2-5, swirl, Gaussians; regrid every 2 coarse steps by tagging
    |grad q|; multirate through the persistent kernel between regrids."""
    from paper_1703_03116_amd.amr import run_adaptive
    gp = S.gaussian_params(3)
    L = S.refine_where(lambda l, ix, iy: S.gaussian_grad_max(gp, (l, ix, iy)) / (mx << l) > 0.02, 2, 4)
    q0 = S.sample_on_leaves(S.gaussians(gp), L, mx)
    ps = B.PatchStore(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), min_level=2, max_level=5,
                      capacity=4 ** 5)
    ps.set_interior(q0)
    o = O.Oracle(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), lmin=2, lmax=5)
    o.set_interior(q0)
    dt = 0.9 / (mx * 4)
    tau_r, tau_c = 2.0, 1.0
    run_adaptive(ps, dt, 6, regrid_every=2, tau_refine=tau_r, tau_coarsen=tau_c)
    _oracle_run_adaptive(o, dt, 6, 2, tau_r, tau_c)
    ps.check()
    assert np.array_equal(np.sort(ps.leaves().view("i4,i4,i4"), axis=0), np.sort(o.leaves().view("i4,i4,i4"), axis=0))
    assert ps.nleaves == o.n and ps.nleaves != len(L)
    assert rel(ps.interior(), o.interior()) <= TOL


def test_full_size_dam_break_levels_2_6(B, O):
    """The dam-break workload at its full size (levels 2-6, 685 patches of
    16x16, reflecting walls, 31 level-steps per coarse step), graph form,
    5 coarse steps, against the oracle."""
    w = S.workload("dam_break")
    ps = B.from_workload(w)
    o = O.from_workload(w)
    dt = 0.6 / (w["mx"] << w["lmin"]) / 2.5  # finest-level Courant number <= 0.6 for |u| + c <= 2.5
    ps.coarse_steps(dt, 5, "graph")
    for s_ in range(5):
        o.coarse_step(s_ * dt, dt)
    ps.check()
    assert rel(ps.interior(), o.interior()) <= TOL


def test_full_size_adaptive_swirl_levels_3_7(B, O):
    """The adaptive workload at its full size (levels 3-7, 8224 patches of
    32x32 at the start), regrid every 2 coarse steps with the bench's
    thresholds, 4 coarse steps: the leaf sets must agree exactly and the
    solution to the tolerance."""
    from paper_1703_03116_amd.amr import run_adaptive
    w = S.workload("swirl_amr")
    ps = B.from_workload(w, capacity=4 ** w["lmax"])
    o = O.from_workload(w)
    dt = w["dt_coarse"]
    run_adaptive(ps, dt, 4, regrid_every=2, tau_refine=0.05, tau_coarsen=0.025)
    _oracle_run_adaptive(o, dt, 4, 2, 0.05, 0.025)
    ps.check()
    assert np.array_equal(np.sort(ps.leaves().view("i4,i4,i4"), axis=0), np.sort(o.leaves().view("i4,i4,i4"), axis=0))
    assert rel(ps.interior(), o.interior()) <= TOL

