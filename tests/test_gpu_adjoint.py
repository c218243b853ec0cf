"""Adjoint of advance + ghost fill on the GPU against the oracle's
hand-written discrete adjoint, and against central finite differences.

MC-limited steps are piecewise linear, so a finite difference crosses
limiter kinks whenever a branch decision sits within eps of a switch.  The
adjoint is pinned exactly against the oracle's discrete adjoint (<= 1e-12
relative); the 1e-6 finite-difference bar is checked for Lax-Wendroff (a
linear map) and for MC on data without flat regions, with the limiter
branch decisions of the two perturbed trajectories compared edge by edge
at every step: where no decision differs, the segment [q - eps d, q + eps d]
lies in one linear piece and central differences are exact up to rounding.
"""
import numpy as np
import pytest

from workloads import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_1703_03116_amd import binding
    binding.lib()
    return binding


def rel(a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("limiter", ["mc", "lw", "minmod"])
@pytest.mark.parametrize("level,mx", [(0, 16), (1, 32), (2, 16), (3, 8)])
def test_adjoint_step_matches_oracle(B, oracle_lib, limiter, level, mx):
    L = S.uniform_leaves(level)
    q = S.sample_on_leaves(lambda x, y: np.exp(-((x - 0.4) ** 2 + (y - 0.6) ** 2) / 0.02)
                           + 0.3 * np.sin(2 * np.pi * x), L, mx)
    lam = np.random.default_rng(level).standard_normal(q.shape)
    ps = B.PatchStore(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter=limiter)
    o = oracle_lib.Oracle(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter=limiter)
    dt = 0.9 / (mx << level)
    g = ps.adjoint_step(level, 0.17, dt, q, lam)
    r = o.adjoint_step(level, 0.17, dt, q, lam)
    assert rel(g, r) <= 1e-12


@pytest.mark.parametrize("limiter", ["mc", "lw", "first", "minmod"])
@pytest.mark.parametrize("level,mx", [(0, 16), (1, 32), (2, 16), (3, 8)])
def test_leaf_order_step_equals_graph_step_bitwise(B, limiter, level, mx):
    """fc_step_uniform (leaf order in and out) reproduces the store's
    graph-mode steps bit for bit, at the times the store accumulates."""
    import torch
    L = S.uniform_leaves(level)
    q0 = torch.tensor(S.sample_on_leaves(S.gaussians(S.gaussian_params(5)), L, mx), device="cuda")
    ps = B.PatchStore(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter=limiter)
    dt = 0.9 / (mx << level)
    ps.time = 0.05
    ps.set_interior(q0)
    q, t = q0, 0.05
    for _ in range(3):
        q = ps.step_uniform(level, t, dt, q)
        t = t + dt
    ps.coarse_steps(dt, 3, "graph")
    assert torch.equal(q, ps.interior())


def test_leaf_order_step_rejects_adaptive_meshes_and_aliasing(B):
    import torch
    L = S.refine_leaves(S.uniform_leaves(1), [0])
    ps = B.PatchStore(L, mx=8, velocity="swirl", vel_params=(1.0, 0, 0))
    q = torch.zeros((len(L), 1, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        ps.step_uniform(1, 0.0, 0.01, q)
    L = S.uniform_leaves(1)
    ps = B.PatchStore(L, mx=8, velocity="swirl", vel_params=(1.0, 0, 0))
    q = torch.zeros((len(L), 1, 8, 8), dtype=torch.float64, device="cuda")
    from paper_1703_03116_amd import binding
    with pytest.raises(RuntimeError):
        binding._check(binding.lib().fc_step_uniform(ps._h, 1, 0.0, 0.01, binding.C.c_void_p(q.data_ptr()),
                                                      binding.C.c_void_p(q.data_ptr()), binding._stream()))


def test_reverse_sweep_matches_oracle_discrete_adjoint(B, oracle_lib):
    """Whole gradient through 40 MC-limited steps with checkpoints every 8."""
    import torch
    from paper_1703_03116_amd.adjoint import loss_and_grad
    level, mx, n = 3, 16, 40
    L = S.uniform_leaves(level)
    q0 = S.sample_on_leaves(S.gaussians(S.gaussian_params(5)), L, mx)
    qt = S.sample_on_leaves(S.gaussians(S.gaussian_params(6)), L, mx)
    dt = 0.9 / (mx << level)
    ps = B.PatchStore(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0))
    Lg, g = loss_and_grad(ps, torch.tensor(q0, device="cuda"), torch.tensor(qt, device="cuda"), level, dt, n, 8)
    o = oracle_lib.Oracle(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0))
    o.set_interior(q0)
    states, t = [], 0.0
    for k in range(n):
        states.append((t, o.interior()))
        o.coarse_step(t, dt)
        t += dt
    lam = o.interior() - qt
    assert abs(Lg.item() - 0.5 * (lam ** 2).sum()) <= 1e-12 * abs(Lg.item())
    for tk, qk in reversed(states):
        lam = o.adjoint_step(level, tk, dt, qk, lam)
    assert rel(g, lam) <= 1e-12


def test_checkpointing_does_not_change_the_gradient(B):
    import torch
    from paper_1703_03116_amd.adjoint import loss_and_grad
    level, mx, n = 2, 32, 24
    L = S.uniform_leaves(level)
    q0 = torch.tensor(S.sample_on_leaves(S.gaussians(S.gaussian_params(5)), L, mx), device="cuda")
    qt = torch.tensor(S.sample_on_leaves(S.gaussians(S.gaussian_params(6)), L, mx), device="cuda")
    ps = B.PatchStore(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0))
    dt = 0.9 / (mx << level)
    _, g1 = loss_and_grad(ps, q0, qt, level, dt, n, 4)
    _, g2 = loss_and_grad(ps, q0, qt, level, dt, n, n)
    L3, g3 = loss_and_grad(ps, q0, qt, level, dt, n, 1)  # every state resident, no recomputation
    assert torch.equal(g1, g2)
    assert torch.equal(g1, g3)
    assert ps.time == pytest.approx(n * dt, rel=1e-12)


def _fd_check(B, limiter, ndir, tol):
    """Uniform level 6 (4096 patches of 32x32), swirl, 256 steps, checkpoint
    every 16; central differences eps = 1e-6 along smooth seeded directions."""
    import torch
    from paper_1703_03116_amd.adjoint import loss, loss_and_grad
    level, mx, n = 6, 32, 256
    L = S.uniform_leaves(level)
    q0 = torch.tensor(S.sample_on_leaves(S.gaussians(S.gaussian_params(5)), L, mx), device="cuda")
    qt = torch.tensor(S.sample_on_leaves(S.gaussians(S.gaussian_params(6)), L, mx), device="cuda")
    dt = 0.9 / (mx << level)
    ps = B.PatchStore(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter=limiter)
    _, g = loss_and_grad(ps, q0, qt, level, dt, n, 16)
    errs = []
    for d in S.smooth_directions(7, ndir, L, mx):
        d = torch.tensor(d, device="cuda")
        eps = 1e-6
        fd = (loss(ps, q0 + eps * d, qt, dt, n) - loss(ps, q0 - eps * d, qt, dt, n)).item() / (2 * eps)
        ad = (g * d).sum().item()
        errs.append(abs(fd - ad) / abs(ad))
        print(f"{limiter} direction {len(errs)}: fd {fd:.12e} adjoint {ad:.12e} rel {errs[-1]:.2e}", flush=True)
    assert max(errs) <= tol, errs


def test_full_size_gradient_matches_finite_differences_linear_scheme(B):
    _fd_check(B, "lw", 20, 1e-6)


def _mc_branches(W, Wu):
    """MC limiter branch per edge: 0 (W Wu <= 0), 1 half-sum, 2 twice W, 3
    twice the upwind wave (ties to the first)."""
    import torch
    pos = W * Wu > 0
    a, b, c = 0.5 * (W + Wu).abs(), 2 * W.abs(), 2 * Wu.abs()
    br = torch.ones_like(W, dtype=torch.int8)
    mn = a.clone()
    m2 = b < mn
    br[m2] = 2
    mn = torch.where(m2, b, mn)
    br[c < mn] = 3
    return torch.where(pos, br, torch.zeros_like(br))


def _branch_masks(q, level, mx, tm):
    """Limiter branches of every x- and y-edge of a uniform periodic level
    for the swirl field at mid-step time tm (upwind side from the sign of
    the edge velocity; edges where it vanishes are left out)."""
    import math
    import torch
    n, NG = 1 << level, mx << level
    G = q.view(n, n, mx, mx).permute(0, 2, 1, 3).reshape(NG, NG)       # [J][I]
    c = torch.sign(torch.sin(2 * math.pi * (torch.arange(NG, device=q.device, dtype=torch.float64) + 0.5) / NG))
    ct = math.cos(math.pi * tm)
    W = G - torch.roll(G, 1, 1)                   # x-edge I of row J; u ~ sin(2 pi y_J) c(t)
    Wu = torch.where((c[:, None] * ct) > 0, torch.roll(W, 1, 1), torch.roll(W, -1, 1))
    bx = _mc_branches(W, Wu)
    bx[:, 0] = 0                                  # u = 0 on the x = 0 edges
    Wy = G - torch.roll(G, 1, 0)                  # y-edge J of column I; v ~ -sin(2 pi x_I) c(t)
    Wyu = torch.where((-c[None, :] * ct) > 0, torch.roll(Wy, 1, 0), torch.roll(Wy, -1, 0))
    by = _mc_branches(Wy, Wyu)
    by[0, :] = 0
    return bx, by


@pytest.mark.parametrize("eps,tol", [(1e-6, 1e-6), (1e-8, 1e-6), (1e-10, 1e-5)])
def test_full_size_gradient_finite_differences_mc(B, eps, tol):
    """MC at the gradient workload's size (uniform level 6, 4096 patches of
    32x32, swirl, 256 steps, checkpoints every 16) on a Gaussian sum over
    two plane waves (no flat regions): 20 smooth directions, central
    differences from the two perturbed trajectories, which are stepped in
    lockstep while their limiter branches are compared.  The flips per
    direction are printed; at eps = 1e-10 none may occur (every segment in
    one linear piece; the bar there is set by rounding, 1e-10 of the
    state), at the larger eps the few that occur must not move the result
    past 1e-6."""
    import torch
    from paper_1703_03116_amd.adjoint import _times, loss_and_grad
    level, mx, n = 6, 32, 256
    L = S.uniform_leaves(level)
    q0 = torch.tensor(S.sample_on_leaves(S.gaussians_on_waves(S.gaussian_params(5)), L, mx), device="cuda")
    qt = torch.tensor(S.sample_on_leaves(S.gaussians(S.gaussian_params(6)), L, mx), device="cuda")
    dt = 0.9 / (mx << level)
    ps = B.PatchStore(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter="mc")
    _, g = loss_and_grad(ps, q0, qt, level, dt, n, 16)
    times = _times(0.0, dt, n)
    errs, flips = [], []
    for d in S.smooth_directions(7, 20, L, mx):
        d = torch.tensor(d, device="cuda")
        qp, qm = (q0 + eps * d).contiguous(), (q0 - eps * d).contiguous()
        nf = 0
        for s in range(n):
            tm = times[s] + 0.5 * dt
            bpx, bpy = _branch_masks(qp, level, mx, tm)
            bmx, bmy = _branch_masks(qm, level, mx, tm)
            nf += int((bpx != bmx).sum().item() + (bpy != bmy).sum().item())
            qp = ps.step_uniform(level, times[s], dt, qp)
            qm = ps.step_uniform(level, times[s], dt, qm)
        fd = (0.5 * ((qp - qm) * (qp + qm - 2 * qt)).sum()).item() / (2 * eps)
        ad = (g * d).sum().item()
        errs.append(abs(fd - ad) / abs(ad))
        flips.append(nf)
        print(f"mc eps {eps:.0e} direction {len(errs)}: branch flips {nf} fd {fd:.12e} adjoint {ad:.12e} "
              f"rel {errs[-1]:.2e}", flush=True)
    assert max(errs) <= tol, errs
    if eps <= 1e-10:
        assert max(flips) == 0, flips


@pytest.mark.parametrize("limiter", ["mc", "minmod"])
def test_full_size_steps_match_oracle(B, oracle_lib, limiter):
    """The gradient workload's size (uniform level 6, 4096 patches of 32x32):
    one leaf-order forward step and one adjoint step, every element, against
    the oracle's step and hand-written discrete adjoint."""
    import torch
    level, mx = 6, 32
    L = S.uniform_leaves(level)
    q = S.sample_on_leaves(S.gaussians(S.gaussian_params(5)), L, mx)
    lam = np.random.default_rng(6).standard_normal(q.shape)
    dt, t = 0.9 / (mx << level), 0.17
    ps = B.PatchStore(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter=limiter)
    o = oracle_lib.Oracle(L, mx=mx, velocity="swirl", vel_params=(1.0, 0, 0), limiter=limiter)
    qd = torch.tensor(q, device="cuda")
    g = ps.adjoint_step(level, t, dt, qd, torch.tensor(lam, device="cuda"))
    assert rel(g, o.adjoint_step(level, t, dt, q, lam)) <= 1e-12
    f = ps.step_uniform(level, t, dt, qd)
    o.set_interior(q)
    o.coarse_step(t, dt)
    assert rel(f, o.interior()) <= 1e-12
