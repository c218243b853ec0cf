"""ctypes wrapper of the FP64 CPU oracle (fc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the GPU library or its
binding.  Data crosses in leaf order as ``[nleaves][nfields][mx][mx]``
float64 arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

EQ = {"advection": 0, "swe": 1}
BC = {"periodic": 0, "reflect": 1}
VEL = {"none": 0, "constant": 1, "swirl": 2}
LIM = {"mc": 0, "lw": 1, "first": 2, "minmod": 3}
ERR = {"stencil": 1, "unbalanced": 2, "cover": 4, "width": 8, "arg": 16}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-std=gnu11", "-Wall", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip, C.c_int, dp, C.c_double,
                                 C.c_int, C.c_int, C.c_int, ip, ip]
        L.orc_create_brick.restype = C.c_void_p
        L.orc_create_brick.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip, C.c_int, dp, C.c_double,
                                       C.c_int, C.c_int, C.c_int, C.c_int, ip, C.c_int, ip, ip]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_mapping.argtypes = [C.c_void_p, C.c_double]
        L.orc_set_mapping.restype = C.c_int
        L.orc_capacity.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.orc_capacity.restype = C.c_double
        for name in ("orc_set_interior", "orc_get_interior", "orc_get_full", "orc_set_full",
                     "orc_get_old_interior"):
            getattr(L, name).argtypes = [C.c_void_p, dp]
        L.orc_nleaves.argtypes = [C.c_void_p]
        L.orc_leaves.argtypes = [C.c_void_p, ip]
        L.orc_error.argtypes = [C.c_void_p]
        L.orc_clear_error.argtypes = [C.c_void_p]
        L.orc_ghost_fill.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double]
        L.orc_advance_level.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
        L.orc_advance_level.restype = C.c_double
        L.orc_coarse_step.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int]
        L.orc_coarse_step.restype = C.c_double
        L.orc_tag.argtypes = [C.c_void_p, C.c_double, C.c_double, C.POINTER(C.c_byte), dp]
        L.orc_adapt.argtypes = [C.c_void_p, C.POINTER(C.c_byte), ip, C.c_int]
        L.orc_adapt.restype = C.c_int
        L.orc_adapt_smooth.argtypes = [C.c_void_p, C.POINTER(C.c_byte), ip, C.c_int]
        L.orc_adapt_smooth.restype = C.c_int
        L.orc_regrid.argtypes = [C.c_void_p, C.c_int, ip]
        L.orc_regrid.restype = C.c_int
        L.orc_tangent_step.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, dp, dp, dp]
        L.orc_adjoint_step.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, dp, dp, dp]
        L.orc_edge_velocity.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_edge_velocity.restype = C.c_double
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


class OracleError(RuntimeError):
    pass


class Oracle:
    """One leaf set with its patch data, advanced by the plain CPU scheme."""

    def __init__(self, leaves, mx=8, mbc=2, equation="advection", limiter="mc",
                 bc=("periodic",) * 4, velocity="constant", vel_params=(1.0, 0.5, 0.0),
                 gravity=1.0, lmin=None, lmax=None, brick=(1, 1), orient=None, map_alpha=0.0):
        """brick: (nbx, nby) unit blocks (Sec. 2.3); orient: one orientation
        code 0..7 per block, block (bx, by) at bx + nbx * by (None: all 0).
        Leaves are (level, ix, iy) with block (ix >> level, iy >> level) and
        the low bits in the block's own indices.  map_alpha: the mapped grid
        X = (xi, eta) + map_alpha sin(2 pi xi) sin(2 pi eta) (1, 1) (0:
        Cartesian)."""
        L = lib()
        leaves = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 3))
        self.mx, self.mbc, self.N = mx, mbc, mx + 2 * mbc
        self.F = 3 if equation == "swe" else 1
        self.lmin = int(leaves[:, 0].min()) if lmin is None else int(lmin)
        self.lmax = int(leaves[:, 0].max()) if lmax is None else int(lmax)
        bca = np.asarray([BC[b] for b in bc], dtype=np.int32)
        vp = np.asarray(list(vel_params) + [0.0] * (3 - len(vel_params)), dtype=np.float64)
        st = C.c_int(0)
        self.brick = (int(brick[0]), int(brick[1]))
        self.orient = None if orient is None else np.ascontiguousarray(np.asarray(orient, dtype=np.int32).ravel())
        if self.orient is not None and self.orient.size != self.brick[0] * self.brick[1]:
            raise OracleError("one orientation code per block")
        self._h = L.orc_create_brick(mx, mbc, EQ[equation], LIM[limiter], _ip(bca), VEL[velocity], _dp(vp),
                                     float(gravity), self.lmin, self.lmax, self.brick[0], self.brick[1],
                                     None if self.orient is None else _ip(self.orient), len(leaves), _ip(leaves),
                                     C.byref(st))
        self._cfg = (mx, mbc, equation, limiter, tuple(bc), velocity, tuple(vel_params), gravity)
        if st.value:
            L.orc_destroy(self._h)
            self._h = None
            raise OracleError(f"oracle rejected the mesh: status {st.value}")
        if map_alpha != 0.0 and L.orc_set_mapping(self._h, float(map_alpha)):
            L.orc_destroy(self._h)
            self._h = None
            raise OracleError("oracle rejected the mapping")
        self.map_alpha = float(map_alpha)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    # -- data ---------------------------------------------------------
    @property
    def n(self):
        return lib().orc_nleaves(self._h)

    def leaves(self):
        out = np.empty((self.n, 3), dtype=np.int32)
        lib().orc_leaves(self._h, _ip(out))
        return out

    def set_interior(self, q):
        q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(self.n, self.F, self.mx, self.mx))
        lib().orc_set_interior(self._h, _dp(q))

    def interior(self):
        out = np.empty((self.n, self.F, self.mx, self.mx))
        lib().orc_get_interior(self._h, _dp(out))
        return out

    def old_interior(self):
        out = np.empty((self.n, self.F, self.mx, self.mx))
        lib().orc_get_old_interior(self._h, _dp(out))
        return out

    def full(self):
        out = np.empty((self.n, self.F, self.N, self.N))
        lib().orc_get_full(self._h, _dp(out))
        return out

    def set_full(self, q):
        q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(self.n, self.F, self.N, self.N))
        lib().orc_set_full(self._h, _dp(q))

    @property
    def error(self):
        return lib().orc_error(self._h)

    def clear_error(self):
        lib().orc_clear_error(self._h)

    # -- the method ----------------------------------------------------
    def ghost_fill(self, lo=None, hi=None, alpha=1.0):
        lo = self.lmin if lo is None else lo
        hi = self.lmax if hi is None else hi
        lib().orc_ghost_fill(self._h, int(lo), int(hi), float(alpha))

    def advance_level(self, level, t, dt):
        return lib().orc_advance_level(self._h, int(level), float(t), float(dt))

    def coarse_step(self, t, dt, mode="multirate"):
        return lib().orc_coarse_step(self._h, float(t), float(dt), 0 if mode == "multirate" else 1)

    def tag(self, tau_r, tau_c):
        tags = np.zeros(self.n, dtype=np.int8)
        g2 = np.zeros(self.n)
        lib().orc_tag(self._h, float(tau_r), float(tau_c), tags.ctypes.data_as(C.POINTER(C.c_byte)), _dp(g2))
        return tags, g2

    def capacity(self, level, I, J):
        """Area of the mapped level-`level` cell (I, J) over h^2."""
        return lib().orc_capacity(self._h, int(level), int(I), int(J))

    def adapt(self, tags, smooth=False):
        """New leaves from tags (Sec. 4.1); smooth: raise each leaf's target
        level to its neighbours' largest first (smooth refinement, Sec. 4.2)."""
        tags = np.ascontiguousarray(np.asarray(tags, dtype=np.int8))
        cap = 4 * self.n + 64
        out = np.zeros((cap, 3), dtype=np.int32)
        fn = lib().orc_adapt_smooth if smooth else lib().orc_adapt
        cnt = fn(self._h, tags.ctypes.data_as(C.POINTER(C.c_byte)), _ip(out), cap)
        if cnt < 0:
            raise OracleError("adapt overflow")
        return out[:cnt].copy()

    def regrid(self, new_leaves):
        nl = np.ascontiguousarray(np.asarray(new_leaves, dtype=np.int32).reshape(-1, 3))
        st = lib().orc_regrid(self._h, len(nl), _ip(nl))
        if st:
            raise OracleError(f"regrid failed: status {st}")

    def tangent_step(self, level, t, dt, q, d):
        q = np.ascontiguousarray(q, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        out = np.empty_like(q)
        lib().orc_tangent_step(self._h, int(level), float(t), float(dt), _dp(q), _dp(d), _dp(out))
        return out

    def edge_velocity(self, level, direction, I, J, tm):
        """Edge velocity of the scalar step: direction 0 gives u on x-edge I
        of row J, direction 1 gives v on y-edge J of column I (level-`level`
        indices), at time tm."""
        return lib().orc_edge_velocity(self._h, int(level), int(direction), int(I), int(J), float(tm))

    def adjoint_step(self, level, t, dt, q, lam):
        q = np.ascontiguousarray(q, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        out = np.empty_like(q)
        lib().orc_adjoint_step(self._h, int(level), float(t), float(dt), _dp(q), _dp(lam), _dp(out))
        return out


def from_workload(w, limiter="mc"):
    """Oracle set up for a workload dict of workloads.synth, with q0 loaded."""
    o = Oracle(w["leaves"], mx=w["mx"], mbc=w["mbc"], equation=w["equation"], limiter=limiter,
               bc=w["bc"], velocity=w["velocity"], vel_params=w["vel_params"],
               gravity=w.get("gravity", 1.0), lmin=w["lmin"], lmax=w["lmax"])
    o.set_interior(w["q0"])
    return o
