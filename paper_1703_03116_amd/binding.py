"""Thin Python binding of the C ABI in include/fc.h (ctypes).

Argument marshalling only: every step of the path runs in the HIP kernels of
libfcmi.so.  PyTorch supplies the device memory (two patch buffers and the
workspace) and the stream.  There is no CPU fallback: loading fails loudly
when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfcmi.so")

EQ = {"advection": 0, "swe": 1}
BC = {"periodic": 0, "reflect": 1}
VEL = {"none": 0, "constant": 1, "swirl": 2}
LIM = {"mc": 0, "lw": 1, "first": 2, "minmod": 3}
STEP = {"multirate": 0, "global": 1}
MODE = {"per_level": 0, "fused": 1, "graph": 2, "fused_levels": 3, "persistent_graph": 4}

FC_ERRORS = {-1: "FC_ERR_ARG", -2: "FC_ERR_UNBALANCED", -3: "FC_ERR_GHOST_WIDTH", -4: "FC_ERR_HIP",
             -5: "FC_ERR_CFL", -6: "FC_ERR_STATE", -7: "FC_ERR_CAPACITY", -8: "FC_ERR_COVER",
             -9: "FC_ERR_NONFINITE"}

EXPORTS = ["fc_last_error", "fc_patchstore_create", "fc_patchstore_create_brick", "fc_patchstore_destroy", "fc_patchstore_sizes",
           "fc_patchstore_bind", "fc_patchstore_info", "fc_patchstore_leaves", "fc_patchstore_records", "fc_set_interior",
           "fc_get_interior", "fc_get_patches", "fc_ghost_fill", "fc_advance_level",
           "fc_advance_coarse_steps", "fc_advance_adaptive", "fc_advance_level_noalloc", "fc_get_time", "fc_set_time", "fc_tag_refine", "fc_adapt", "fc_adapt_device", "fc_regrid",
           "fc_prepare_steps", "fc_step_uniform", "fc_adjoint_step", "fc_check_device", "fc_autotune", "fc_set_variant", "fc_set_persistent_grid",
           "fc_set_tile", "fc_get_launch"]


class FcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{FC_ERRORS.get(status, status)}: {msg}")
        self.status = status


class Leaf(C.Structure):
    _fields_ = [("level", C.c_int32), ("ix", C.c_int32), ("iy", C.c_int32)]


class Config(C.Structure):
    _fields_ = [("mx", C.c_int32), ("mbc", C.c_int32), ("equation", C.c_int32), ("limiter", C.c_int32),
                ("bc", C.c_int32 * 4), ("velocity", C.c_int32), ("vel_params", C.c_double * 3),
                ("gravity", C.c_double), ("min_level", C.c_int32), ("max_level", C.c_int32),
                ("time_stepping", C.c_int32), ("reserved", C.c_int32), ("capacity", C.c_int64),
                ("cfl_max", C.c_double), ("map_alpha", C.c_double)]


_lib = None


def lib():
    """Load libfcmi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FcError(-6, f"{LIB_PATH} is missing: build it with paper_1703_03116_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.fc_last_error.restype = C.c_char_p
        L.fc_patchstore_create.argtypes = [C.POINTER(Config), C.c_int64, C.POINTER(Leaf), C.POINTER(vp),
                                           C.POINTER(C.c_int64)]
        L.fc_patchstore_create_brick.argtypes = [C.POINTER(Config), C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                                 C.c_int64, C.POINTER(Leaf), C.POINTER(vp), C.POINTER(C.c_int64)]
        L.fc_patchstore_destroy.argtypes = [vp]
        L.fc_patchstore_sizes.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.fc_patchstore_bind.argtypes = [vp, vp, vp, vp, vp]
        L.fc_patchstore_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.fc_patchstore_leaves.argtypes = [vp, C.POINTER(Leaf)]
        L.fc_patchstore_records.argtypes = [vp, C.POINTER(C.c_int32)]
        for f in ("fc_set_interior", "fc_get_interior", "fc_get_patches"):
            getattr(L, f).argtypes = [vp, vp, vp]
        L.fc_ghost_fill.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, vp]
        L.fc_advance_level.argtypes = [vp, C.c_int32, C.c_double, C.c_double, vp, vp]
        L.fc_advance_level_noalloc.argtypes = [vp, C.c_int32, C.c_double, C.c_double, vp, vp]
        L.fc_advance_coarse_steps.argtypes = [vp, C.c_double, C.c_int32, C.c_int32, vp, vp]
        L.fc_advance_adaptive.argtypes = [vp, C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                          C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp]
        L.fc_get_time.argtypes = [vp, C.POINTER(C.c_double)]
        L.fc_set_time.argtypes = [vp, C.c_double]
        L.fc_tag_refine.argtypes = [vp, C.c_double, C.c_double, vp, vp, vp]
        L.fc_adapt.argtypes = [vp, C.POINTER(C.c_int8), C.c_int32, C.POINTER(Leaf), C.c_int64, C.POINTER(C.c_int64)]
        L.fc_adapt_device.argtypes = [vp, vp, C.c_int32, C.POINTER(Leaf), C.c_int64, C.POINTER(C.c_int64), vp]
        L.fc_regrid.argtypes = [vp, C.c_int64, C.POINTER(Leaf), vp]
        L.fc_prepare_steps.argtypes = [vp, C.c_double, C.c_int32, C.c_int32, vp]
        L.fc_step_uniform.argtypes = [vp, C.c_int32, C.c_double, C.c_double, vp, vp, vp]
        L.fc_adjoint_step.argtypes = [vp, C.c_int32, C.c_double, C.c_double, vp, vp, vp, vp]
        L.fc_check_device.argtypes = [vp, vp]
        L.fc_autotune.argtypes = [vp, C.POINTER(C.c_int32), vp]
        L.fc_set_tile.argtypes = [vp, C.c_int32]
        L.fc_get_launch.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.fc_set_variant.argtypes = [vp, C.c_int32]
        L.fc_set_persistent_grid.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
        for f in EXPORTS:
            if f != "fc_last_error":
                getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise FcError(st, lib().fc_last_error().decode())


def _leaves_array(leaves):
    a = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 3))
    arr = (Leaf * len(a))()
    C.memmove(arr, a.ctypes.data, a.nbytes)
    return arr, len(a)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype=torch.float64):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t))
    return t.to(device="cuda", dtype=dtype).contiguous()


class PatchStore:
    """A quadtree leaf set with its patch data resident in HBM."""

    def __init__(self, leaves, mx=32, equation="advection", limiter="mc", bc=("periodic",) * 4,
                 velocity="swirl", vel_params=(1.0, 0.0, 0.0), gravity=1.0, min_level=None, max_level=None,
                 time_stepping="multirate", capacity=None, cfl_max=0.0, brick=(1, 1), orient=None,
                 map_alpha=0.0):
        """brick, orient: a multiblock brick of brick[0] x brick[1] unit
        blocks with one orientation code per block (fc_patchstore_create_brick);
        leaves then lie in the blocks' own coordinates.  map_alpha: the
        amplitude of the mapped grid (0: Cartesian)."""
        L = lib()
        arr, n = _leaves_array(leaves)
        lv = np.asarray(leaves, dtype=np.int32).reshape(-1, 3)
        cfg = Config()
        cfg.mx, cfg.mbc = mx, 2
        cfg.equation, cfg.limiter = EQ[equation], LIM[limiter]
        for s in range(4):
            cfg.bc[s] = BC[bc[s]]
        cfg.velocity = VEL[velocity]
        vp = list(vel_params) + [0.0] * (3 - len(vel_params))
        for s in range(3):
            cfg.vel_params[s] = float(vp[s])
        cfg.gravity = float(gravity)
        cfg.min_level = int(lv[:, 0].min()) if min_level is None else int(min_level)
        cfg.max_level = int(lv[:, 0].max()) if max_level is None else int(max_level)
        cfg.time_stepping = STEP[time_stepping]
        cfg.capacity = int(capacity if capacity is not None else n)
        cfg.cfl_max = float(cfl_max)
        cfg.map_alpha = float(map_alpha)
        self.cfg = cfg
        self.mx, self.N, self.F = mx, mx + 4, 3 if equation == "swe" else 1
        self.min_level, self.max_level = cfg.min_level, cfg.max_level
        h = C.c_void_p()
        perm = (C.c_int64 * n)()
        ori = None
        if orient is not None:
            o = np.ascontiguousarray(np.asarray(orient, dtype=np.int32).ravel())
            ori = (C.c_int32 * len(o))(*o.tolist())
        self.brick = (int(brick[0]), int(brick[1]))
        _check(L.fc_patchstore_create_brick(C.byref(cfg), self.brick[0], self.brick[1], ori, n, arr, C.byref(h),
                                            perm))
        self._h = h
        self.perm = np.frombuffer(perm, dtype=np.int64).copy()
        qd, wb = C.c_int64(), C.c_int64()
        _check(L.fc_patchstore_sizes(h, C.byref(qd), C.byref(wb)))
        dev = torch.device("cuda")
        self.q0 = torch.zeros(qd.value, dtype=torch.float64, device=dev)
        self.q1 = torch.zeros(qd.value, dtype=torch.float64, device=dev)
        self.ws = torch.zeros(wb.value + 256, dtype=torch.uint8, device=dev)
        off = (-self.ws.data_ptr()) % 256
        self._ws_ptr = self.ws.data_ptr() + off
        _check(L.fc_patchstore_bind(h, C.c_void_p(self.q0.data_ptr()), C.c_void_p(self.q1.data_ptr()),
                                    C.c_void_p(self._ws_ptr), _stream()))
        self.nleaves = n
        self.input_leaves = lv.copy()   # the order interior arrays use

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.fc_patchstore_destroy(h)
            self._h = None

    # -- data ---------------------------------------------------------------
    def leaves(self):
        """Store-order leaves."""
        out = (Leaf * self.nleaves)()
        _check(lib().fc_patchstore_leaves(self._h, out))
        return np.array([(x.level, x.ix, x.iy) for x in out], dtype=np.int32)

    def set_interior(self, q):
        q = _dev(q).reshape(self.nleaves, self.F, self.mx, self.mx)
        self._keep = q
        _check(lib().fc_set_interior(self._h, C.c_void_p(q.data_ptr()), _stream()))

    def interior(self):
        out = torch.empty((self.nleaves, self.F, self.mx, self.mx), dtype=torch.float64, device="cuda")
        _check(lib().fc_get_interior(self._h, C.c_void_p(out.data_ptr()), _stream()))
        return out

    def patches(self):
        out = torch.empty((self.nleaves, self.F, self.N, self.N), dtype=torch.float64, device="cuda")
        _check(lib().fc_get_patches(self._h, C.c_void_p(out.data_ptr()), _stream()))
        return out

    @property
    def time(self):
        t = C.c_double()
        _check(lib().fc_get_time(self._h, C.byref(t)))
        return t.value

    @time.setter
    def time(self, t):
        _check(lib().fc_set_time(self._h, float(t)))

    # -- the method ---------------------------------------------------------
    def ghost_fill(self, lo=None, hi=None, alpha=1.0):
        lo = self.min_level if lo is None else lo
        hi = self.max_level if hi is None else hi
        _check(lib().fc_ghost_fill(self._h, int(lo), int(hi), float(alpha), _stream()))

    def advance_level(self, level, t, dt, cfl=None):
        p = C.c_void_p(cfl.data_ptr()) if cfl is not None else None
        _check(lib().fc_advance_level(self._h, int(level), float(t), float(dt), p, _stream()))

    def prepare_steps(self, dt_coarse, nsteps, mode="graph"):
        """Capture the graphs the next coarse_steps(dt_coarse, nsteps, mode)
        replays (one-time set-up kept out of that call)."""
        _check(lib().fc_prepare_steps(self._h, float(dt_coarse), int(nsteps), MODE[mode], _stream()))

    def coarse_steps(self, dt_coarse, nsteps=1, mode="per_level", cfl=None):
        p = C.c_void_p(cfl.data_ptr()) if cfl is not None else None
        _check(lib().fc_advance_coarse_steps(self._h, float(dt_coarse), int(nsteps), MODE[mode], p, _stream()))

    def advance_adaptive(self, t_end, dt, cfl_target=0.9, mode="graph", max_steps=100000):
        """Clawpack-style adaptive coarse steps to t_end (needs cfl_max at
        creation); returns (next proposed dt, accepted steps, rejected steps)."""
        d = C.c_double(float(dt))
        ns, nr = C.c_int32(), C.c_int32()
        _check(lib().fc_advance_adaptive(self._h, float(t_end), float(cfl_target), MODE[mode], C.byref(d),
                                         int(max_steps), C.byref(ns), C.byref(nr), _stream()))
        return d.value, ns.value, nr.value

    def tag(self, tau_refine, tau_coarsen):
        tags = torch.zeros(self.nleaves, dtype=torch.int8, device="cuda")
        g2 = torch.zeros(self.nleaves, dtype=torch.float64, device="cuda")
        _check(lib().fc_tag_refine(self._h, float(tau_refine), float(tau_coarsen), C.c_void_p(tags.data_ptr()),
                                   C.c_void_p(g2.data_ptr()), _stream()))
        return tags, g2

    def adapt(self, tags, smooth=False):
        """New leaves from tags, adapted on the host (smooth: Sec. 4.2)."""
        t = np.ascontiguousarray(np.asarray(tags.cpu() if isinstance(tags, torch.Tensor) else tags, dtype=np.int8))
        cap = 4 * self.nleaves + 64
        out = (Leaf * cap)()
        n = C.c_int64()
        _check(lib().fc_adapt(self._h, t.ctypes.data_as(C.POINTER(C.c_int8)), int(bool(smooth)), out, cap, C.byref(n)))
        return np.frombuffer(out, dtype=np.int32, count=3 * n.value).reshape(-1, 3).copy()

    def adapt_device(self, tags, smooth=False):
        """The same adaptation on the device from device tags (as tag()
        returns them); only the new leaf list comes back."""
        t = _dev(tags, torch.int8)
        cap = max(4 * self.nleaves + 64, int(self.cfg.capacity))
        out = (Leaf * cap)()
        n = C.c_int64()
        _check(lib().fc_adapt_device(self._h, C.c_void_p(t.data_ptr()), int(bool(smooth)), out, cap, C.byref(n),
                                     _stream()))
        return np.frombuffer(out, dtype=np.int32, count=3 * n.value).reshape(-1, 3).copy()

    def regrid(self, new_leaves):
        arr, n = _leaves_array(new_leaves)
        _check(lib().fc_regrid(self._h, n, arr, _stream()))
        self.nleaves = n
        self.input_leaves = np.asarray(new_leaves, dtype=np.int32).reshape(-1, 3).copy()

    def step_uniform(self, level, t, dt, q_in):
        """q(t + dt) from q(t) = q_in on a uniform periodic level, leaf order;
        the store's own state is not touched."""
        q = _dev(q_in).reshape(self.nleaves, 1, self.mx, self.mx)
        out = torch.empty_like(q)
        _check(lib().fc_step_uniform(self._h, int(level), float(t), float(dt), C.c_void_p(q.data_ptr()),
                                     C.c_void_p(out.data_ptr()), _stream()))
        return out

    def adjoint_step(self, level, t, dt, q_in, lam_in):
        q = _dev(q_in).reshape(self.nleaves, 1, self.mx, self.mx)
        lam = _dev(lam_in).reshape(self.nleaves, 1, self.mx, self.mx)
        out = torch.empty_like(lam)
        _check(lib().fc_adjoint_step(self._h, int(level), float(t), float(dt), C.c_void_p(q.data_ptr()),
                                     C.c_void_p(lam.data_ptr()), C.c_void_p(out.data_ptr()), _stream()))
        return out

    def check(self):
        _check(lib().fc_check_device(self._h, _stream()))

    def autotune(self):
        nt = C.c_int32()
        _check(lib().fc_autotune(self._h, C.byref(nt), _stream()))
        return nt.value

    def set_variant(self, threads_per_patch):
        _check(lib().fc_set_variant(self._h, int(threads_per_patch)))

    def set_tile(self, seg_cells=0):
        """Cells per sweep segment of the scalar advance (0: the default)."""
        _check(lib().fc_set_tile(self._h, int(seg_cells)))

    def launch(self):
        """(threads per patch, cells per sweep segment) in use."""
        nt, sg = C.c_int32(), C.c_int32()
        _check(lib().fc_get_launch(self._h, C.byref(nt), C.byref(sg)))
        return nt.value, sg.value

    def set_persistent_grid(self, grid=0):
        """Persistent-kernel workgroups (0: all that fit); returns the maximum."""
        mg = C.c_int32()
        _check(lib().fc_set_persistent_grid(self._h, int(grid), C.byref(mg)))
        return mg.value


def from_workload(w, limiter="mc", capacity=None, time_stepping=None, cfl_max=0.0):
    """PatchStore for a workloads.synth workload dict, q0 loaded."""
    ps = PatchStore(w["leaves"], mx=w["mx"], equation=w["equation"], limiter=limiter, bc=w["bc"],
                    velocity=w["velocity"], vel_params=w["vel_params"], gravity=w.get("gravity", 1.0),
                    min_level=w["lmin"], max_level=w["lmax"],
                    time_stepping=time_stepping or w.get("time_stepping", "multirate"), capacity=capacity,
                    cfl_max=cfl_max)
    ps.set_interior(w["q0"])
    return ps
