"""Adjoint of advance + ghost fill on the GPU against the oracle's
hand-written discrete adjoint, and against central finite differences.

MC-limited steps are piecewise linear, so a finite difference crosses
limiter kinks whenever a branch decision sits within eps of a switch; exact
agreement is therefore pinned against the oracle's discrete adjoint
(<= 1e-12 relative), while the 1e-6 finite-difference bar is checked where
the map is linear (Lax-Wendroff), and the MC finite-difference error is
bounded loosely.
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


def test_full_size_gradient_finite_differences_mc(B):
    _fd_check(B, "mc", 6, 5e-2)


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
