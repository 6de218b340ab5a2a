"""Plain FP64 CPU oracle of the successive-convolution fast summation.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_2007_03041_amd``); the arithmetic lives in ``sc_oracle.c`` (plain loops, FP64,
``-O2 -ffp-contract=off``), and this module only marshals numpy arrays into it.

Paper: Christlieb, Guthrey, Sands, Thavappiragasm (2020), "Parallel Algorithms for Successive
Convolution".  Section references are given on each function of ``sc_oracle.c``.

Array convention: numpy arrays in C order with shape ``(n[ndim-1], ..., n[0])`` -- axis 0 of the
grid (x) is the last, contiguous numpy axis.  Periodic axes store ``n`` points with
``dx = (hi-lo)/n``; Dirichlet axes store both ends with ``dx = (hi-lo)/(n-1)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from ctypes import POINTER, c_double, c_int, c_int32, c_int64

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OP_L, OP_R, OP_0 = 0, 1, 2
BC_PERIODIC, BC_DIRICHLET = 0, 1
_OPS = {"L": OP_L, "R": OP_R, "0": OP_0, 0: OP_L, 1: OP_R, 2: OP_0}
_BCS = {"periodic": BC_PERIODIC, "dirichlet": BC_DIRICHLET, 0: BC_PERIODIC, 1: BC_DIRICHLET}


NATIVE_LIB_PATH = os.path.join(_HERE, "liboracle_native.so")
REFERENCE_FLAGS = ["-O2", "-ffp-contract=off"]
NATIVE_FLAGS = ["-O3", "-march=native"]


def build() -> str:
    """Compile the oracle with gcc (plain C, OpenMP over independent lines)."""
    cmd = ["gcc", *REFERENCE_FLAGS, "-fopenmp", "-shared", "-fPIC", "-o", LIB_PATH, _SRC, "-lm"]
    subprocess.check_call(cmd, cwd=_HERE)
    return LIB_PATH


def build_native() -> str:
    """A second build of the same source with ``-O3 -march=native`` (contraction allowed), for CPU
    timing only: every test checks results of the reference build."""
    cmd = ["gcc", *NATIVE_FLAGS, "-fopenmp", "-shared", "-fPIC", "-o", NATIVE_LIB_PATH, _SRC, "-lm"]
    subprocess.check_call(cmd, cwd=_HERE)
    return NATIVE_LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", c_int32), ("n", c_int64 * 3), ("lo", c_double * 3),
                ("hi", c_double * 3), ("bc", c_int32 * 3)]


class _Pde(ctypes.Structure):
    _fields_ = [("c", c_double * 3), ("nu_diff", c_double), ("beta", c_double),
                ("dt", c_double), ("order", c_int32), ("split", c_int32)]


_lib = None
_libs = {}
_build_kind = "reference"


def use_build(kind: str) -> None:
    """Route every call of this module to the ``reference`` build (``-O2 -ffp-contract=off``, the
    default) or the ``native`` timing build (``-O3 -march=native``)."""
    global _lib, _build_kind
    if kind not in ("reference", "native"):
        raise ValueError("build kind: reference or native")
    _build_kind = kind
    _lib = _libs.get(kind)


def set_threads(n: int) -> int:
    """Threads of the loops over lines in the current build; returns the count now in effect."""
    return int(_load().sco_set_threads(int(n)))


def _load():
    global _lib
    if _lib is None:
        path = LIB_PATH if _build_kind == "reference" else NATIVE_LIB_PATH
        override = os.environ.get("SC_ORACLE_LIBRARY_PATH")  # e.g. a sanitizer build (tests)
        if override and _build_kind == "reference":
            path = override
        elif not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build() if _build_kind == "reference" else build_native()
        lib = ctypes.CDLL(path)
        dp = POINTER(c_double)
        lib.sco_weights.argtypes = [c_double, c_int, POINTER(c_int), dp]
        lib.sco_line_quad.argtypes = [c_int, c_int, c_double, c_double, c_int64, dp, dp, dp]
        lib.sco_line_sweep.argtypes = [c_int, c_double, c_double, c_int64, dp, dp, dp, dp, dp]
        lib.sco_line_invL.argtypes = [c_int, c_int, c_int, c_double, c_double, c_int64, dp,
                                      c_double, c_double, dp]
        gp = POINTER(_Grid)
        lib.sco_local_quad.argtypes = [gp, c_int, c_int, c_double, dp, dp, dp]
        lib.sco_sweep_LR.argtypes = [gp, c_int, c_double, dp, dp, dp, dp, dp]
        lib.sco_apply_invL.argtypes = [gp, c_int, c_int, c_int, c_double, dp, dp, dp]
        lib.sco_apply_D_partial_sum.argtypes = [gp, c_int, c_int, c_int, c_double, c_int,
                                                c_double, dp, dp, dp]
        lib.sco_time_step.argtypes = [gp, POINTER(_Pde), c_int, dp]
        lib.sco_line_invL_nn.argtypes = [c_int, c_int, c_int, c_double, c_double, c_int64, c_int64, dp,
                                         c_double, c_double, dp]
        lib.sco_apply_invL_nn.argtypes = [gp, c_int, c_int, c_int, c_double, c_int64, dp, dp, dp]
        lib.sco_num_threads.argtypes = []
        lib.sco_set_threads.argtypes = [c_int]
        for f in ("sco_weights", "sco_line_quad", "sco_line_sweep", "sco_line_invL",
                  "sco_local_quad", "sco_sweep_LR", "sco_apply_invL",
                  "sco_apply_D_partial_sum", "sco_time_step", "sco_num_threads", "sco_set_threads",
                  "sco_line_invL_nn", "sco_apply_invL_nn"):
            getattr(lib, f).restype = c_int
        _libs[_build_kind] = lib
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def make_grid(n, lo=None, hi=None, bc=None) -> _Grid:
    """n: tuple (n0[, n1[, n2]]) with n0 = x (contiguous)."""
    n = tuple(int(v) for v in n)
    nd = len(n)
    lo = tuple(lo) if lo is not None else (0.0,) * nd
    hi = tuple(hi) if hi is not None else (1.0,) * nd
    bc = tuple(_BCS[b] for b in bc) if bc is not None else (BC_PERIODIC,) * nd
    g = _Grid()
    g.ndim = nd
    for e in range(3):
        g.n[e] = n[e] if e < nd else 1
        g.lo[e] = lo[e] if e < nd else 0.0
        g.hi[e] = hi[e] if e < nd else 1.0
        g.bc[e] = bc[e] if e < nd else BC_PERIODIC
    return g


def num_threads() -> int:
    return int(_load().sco_num_threads())


def weights(nu: float, eta) -> np.ndarray:
    """w_j = nu * int_0^1 e^{-nu eta} l_j(eta) d eta on the integer nodes ``eta``."""
    eta = list(int(e) for e in eta)
    arr = (c_int * len(eta))(*eta)
    w = np.zeros(len(eta))
    _check(_load().sco_weights(float(nu), len(eta), arr, _p(w)), "weights")
    return w


def line_quad(bc, order, alpha, dx, v):
    v = _f64(v)
    JL, JR = np.zeros_like(v), np.zeros_like(v)
    _check(_load().sco_line_quad(_BCS[bc], order, alpha, dx, v.size, _p(v), _p(JL), _p(JR)),
           "line_quad")
    return JL, JR


def line_sweep(bc, alpha, dx, JL, JR):
    JL, JR = _f64(JL), _f64(JR)
    IL, IR, ends = np.zeros_like(JL), np.zeros_like(JL), np.zeros(2)
    _check(_load().sco_line_sweep(_BCS[bc], alpha, dx, JL.size, _p(JL), _p(JR), _p(IL), _p(IR),
                                  _p(ends)), "line_sweep")
    return IL, IR, ends


def line_invL(bc, op, order, alpha, dx, v, ga=0.0, gb=0.0):
    v = _f64(v)
    out = np.zeros_like(v)
    _check(_load().sco_line_invL(_BCS[bc], _OPS[op], order, alpha, dx, v.size, _p(v), ga, gb,
                                 _p(out)), "line_invL")
    return out


def _gvals(g, lines):
    if g is None:
        return None
    g = _f64(g).reshape(-1)
    if g.size != 2 * lines:
        raise ValueError("Dirichlet values need 2 per line")
    return g


def local_quad(grid: _Grid, dim, order, alpha, v):
    v = _f64(v)
    JL, JR = np.zeros_like(v), np.zeros_like(v)
    _check(_load().sco_local_quad(ctypes.byref(grid), dim, order, alpha, _p(v), _p(JL), _p(JR)),
           "local_quad")
    return JL, JR


def sweep_LR(grid: _Grid, dim, alpha, JL, JR):
    JL, JR = _f64(JL), _f64(JR)
    IL, IR = np.zeros_like(JL), np.zeros_like(JL)
    lines = JL.size // grid.n[dim]
    ends = np.zeros((lines, 2))
    _check(_load().sco_sweep_LR(ctypes.byref(grid), dim, alpha, _p(JL), _p(JR), _p(IL), _p(IR),
                                _p(ends)), "sweep_LR")
    return IL, IR, ends


def apply_invL(grid: _Grid, dim, op, order, alpha, v, g=None):
    v = _f64(v)
    out = np.zeros_like(v)
    gv = _gvals(g, v.size // grid.n[dim])
    _check(_load().sco_apply_invL(ctypes.byref(grid), dim, _OPS[op], order, alpha,
                                  _p(gv) if gv is not None else None, _p(v), _p(out)),
           "apply_invL")
    return out


def line_invL_nn(bc, op, order, alpha, dx, v, block, ga=0.0, gb=0.0):
    """Nearest-neighbour block form of line_invL (Sec. 3): blocks of `block` points."""
    v = _f64(v)
    out = np.zeros_like(v)
    _check(_load().sco_line_invL_nn(_BCS[bc], _OPS[op], order, alpha, dx, v.size, int(block), _p(v), ga, gb,
                                    _p(out)), "line_invL_nn")
    return out


def apply_invL_nn(grid: _Grid, dim, op, order, alpha, v, block, g=None):
    """line_invL_nn along every line of axis `dim` (blocks of `block` points)."""
    v = _f64(v)
    out = np.zeros_like(v)
    gv = _gvals(g, v.size // grid.n[dim])
    _check(_load().sco_apply_invL_nn(ctypes.byref(grid), dim, _OPS[op], order, alpha, int(block),
                                     _p(gv) if gv is not None else None, _p(v), _p(out)),
           "apply_invL_nn")
    return out


def apply_D_partial_sum(grid: _Grid, dim, op, order, alpha, k, scale, v, g=None):
    v = _f64(v)
    out = np.zeros_like(v)
    gv = _gvals(g, v.size // grid.n[dim])
    _check(_load().sco_apply_D_partial_sum(ctypes.byref(grid), dim, _OPS[op], order, alpha, k,
                                           scale, _p(gv) if gv is not None else None, _p(v),
                                           _p(out)), "apply_D_partial_sum")
    return out


def time_step(grid: _Grid, c, nu_diff, beta, dt, order, nsteps, u, split=False):
    u = _f64(u).copy()
    p = _Pde()
    for e in range(3):
        p.c[e] = c[e] if e < len(c) else 0.0
    p.nu_diff, p.beta, p.dt, p.order, p.split = nu_diff, beta, dt, order, int(bool(split))
    _check(_load().sco_time_step(ctypes.byref(grid), ctypes.byref(p), nsteps, _p(u)),
           "time_step")
    return u


def _euler_partial_sums(grid: _Grid, c, nu_diff, beta, dt, order, u, k):
    """u + dt F(u), F the right-hand side of u_t + c.grad u = nu lap u with every D replaced by the
    partial sum S_k = sum_{p=1..k} D^p (Sec. 2.5): -|c_d| dt alpha S_k(D_{R/L}) - nu dt alpha^2 S_k(D_0)."""
    import math

    out = u.copy()
    for dim in range(grid.ndim):
        cd = c[dim] if dim < len(c) else 0.0
        if cd != 0.0:
            a = beta / (abs(cd) * dt)
            out += -abs(cd) * dt * a * apply_D_partial_sum(grid, dim, "R" if cd > 0 else "L", order, a, k, 1.0, u)
        if nu_diff > 0.0:
            a = beta / math.sqrt(nu_diff * dt)
            out += -nu_diff * dt * a * a * apply_D_partial_sum(grid, dim, "0", order, a, k, 1.0, u)
    return out


def time_step_rk(grid: _Grid, c, nu_diff, beta, dt, order, nsteps, u, stages):
    """s-stage explicit Runge-Kutta (Sec. 2.5) coupled to partial sums of the same order s, in the
    strong-stability-preserving Shu-Osher forms (s = 1: forward Euler; s = 2: u1 = E(u),
    u <- u/2 + E(u1)/2; s = 3: u1 = E(u), u2 = 3u/4 + E(u1)/4, u <- u/3 + 2 E(u2)/3), E the Euler
    step with S_s.  Periodic axes only (partial sums beyond k = 1 need periodic lines)."""
    u = _f64(u).copy()

    def E(v):
        return _euler_partial_sums(grid, c, nu_diff, beta, dt, order, v, stages)

    for _ in range(nsteps):
        if stages == 1:
            u = E(u)
        elif stages == 2:
            u1 = E(u)
            u = 0.5 * u + 0.5 * E(u1)
        elif stages == 3:
            u1 = E(u)
            u2 = 0.75 * u + 0.25 * E(u1)
            u = u / 3.0 + (2.0 / 3.0) * E(u2)
        else:
            raise ValueError("stages must be 1, 2 or 3")
    return u
