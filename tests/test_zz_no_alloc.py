"""The allocation-free entry point fc_advance_level_noalloc, called through
the C ABI: bitwise the step of fc_advance_level, with the same Courant
number, on two calls in a row on one GPU, the second with a smaller store
(the fixed scratch array keeps the first call's larger contents); and its
capacity limit, checked on the host before any device work."""
import ctypes as C

import numpy as np
import pytest

from workloads import synth as S


@pytest.fixture(scope="module")
def B():
    from paper_1703_03116_amd import binding
    binding.lib()
    return binding


@pytest.mark.gpu
def test_no_alloc_step_equals_advance_level_on_two_calls(B):
    import torch
    assert torch.cuda.is_available(), "GPU test"
    L = B.lib()
    for level, mx in ((5, 32), (2, 16)):          # 1024 patches, then 16
        w = S.workload("swirl_uniform", level=level, mx=mx)
        a, b = B.from_workload(w), B.from_workload(w)
        ca = torch.zeros(1, dtype=torch.float64, device="cuda")
        cb = torch.zeros(1, dtype=torch.float64, device="cuda")
        dt = w["dt_coarse"]
        for step in range(2):
            t = 0.1 + step * dt
            a.ghost_fill()
            b.ghost_fill()
            a.advance_level(level, t, dt, ca)
            st = L.fc_advance_level_noalloc(b._h, level, t, dt, C.c_void_p(cb.data_ptr()), B._stream())
            assert st == 0, L.fc_last_error()
        b.check()
        assert torch.equal(a.interior(), b.interior())
        assert ca.item() == cb.item() and 0.5 < cb.item() <= 0.9
    # without a Courant number the scratch array is not touched at all
    w = S.workload("swirl_uniform", level=2, mx=8)
    a, b = B.from_workload(w), B.from_workload(w)
    a.ghost_fill()
    b.ghost_fill()
    a.advance_level(2, 0.0, w["dt_coarse"])
    assert L.fc_advance_level_noalloc(b._h, 2, 0.0, w["dt_coarse"], None, B._stream()) == 0
    assert torch.equal(a.interior(), b.interior())


def test_no_alloc_rejects_stores_beyond_the_scratch_array(B):
    """Capacity above 65536 slots: FC_ERR_CAPACITY before anything else (no
    GPU needed; the store is not even bound)."""
    L = B.lib()
    cfg = B.Config()
    cfg.mx, cfg.mbc, cfg.equation, cfg.limiter = 8, 2, 0, 0
    cfg.velocity = 1
    cfg.vel_params[0] = 1.0
    cfg.min_level, cfg.max_level, cfg.capacity = 0, 9, 70000
    arr, n = B._leaves_array(S.uniform_leaves(1))
    h = C.c_void_p()
    assert L.fc_patchstore_create(C.byref(cfg), n, arr, C.byref(h), None) == 0
    assert L.fc_advance_level_noalloc(h, 1, 0.0, 0.01, None, None) == -7
    assert b"65536" in L.fc_last_error()
    L.fc_patchstore_destroy(h)
