"""MI355X (gfx950) successive-convolution library -- thin Python binding of ``libsc.so``.

This module only marshals arguments: torch tensors supply device memory and the current HIP
stream; every step of the computation runs in the library's HIP kernels (see ``include/sc.h``).
If the library is not built, every entry point raises -- there is no CPU fallback.

Array convention: a grid with ``n = (n0, n1, n2)`` is a contiguous tensor of shape
``(n2, n1, n0)`` (axis 0 = x is the last, contiguous tensor dimension); 1-D and 2-D grids drop the
leading dimensions.  ``dim`` counts grid axes (0 = x).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p
from dataclasses import dataclass, field
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
# SC_LIBRARY_PATH selects another build of the same library (the sanitizer build of the tests)
LIB_PATH = os.environ.get("SC_LIBRARY_PATH") or os.path.join(_HERE, "libsc.so")

SC_OK, SC_ERR_ARG, SC_ERR_SHAPE, SC_ERR_UNSUPPORTED, SC_ERR_WORKSPACE, SC_ERR_DEVICE = 0, -1, -2, -3, -4, -5
SC_F64, SC_F32_MIXED = 0, 1
OPS = {"L": 0, "R": 1, "0": 2}
BCS = {"periodic": 0, "dirichlet": 1}
_STATUS = {0: "SC_OK", -1: "SC_ERR_ARG", -2: "SC_ERR_SHAPE", -3: "SC_ERR_UNSUPPORTED",
           -4: "SC_ERR_WORKSPACE", -5: "SC_ERR_DEVICE"}

# exported symbols of include/sc.h
SYMBOLS = ("sc_local_quad", "sc_sweep_LR", "sc_apply_invL", "sc_apply_D_partial_sum",
           "sc_time_step", "sc_workspace_bytes", "sc_effective_dt", "sc_last_error",
           "sc_timing_enable", "sc_timing_select", "sc_timing_read", "sc_timing_reset",
           "sc_batch_plan_create", "sc_batch_plan_destroy", "sc_batch_workspace_bytes",
           "sc_batch_elements", "sc_batch_apply", "sc_batch_apply_per_instance", "sc_batch_tune",
           "sc_batch_describe", "sc_hj_workspace_bytes", "sc_hj_init", "sc_hj_step", "sc_hj_harvest",
           "sc_mlp_param_count", "sc_mlp_forward", "sc_mlp_grad_workspace_bytes", "sc_mlp_grad", "sc_mlp_adam",
           "sc_apply_invL_noalloc", "sc_apply_invL_nn", "sc_chunk_points", "sc_batch_tune_export",
           "sc_batch_tune_import")
# fixed scratch of sc_apply_invL_noalloc (SC_NOALLOC_SCRATCH_BYTES in include/sc.h)
NOALLOC_SCRATCH_BYTES = 8 << 20


class ScError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class sc_grid(ctypes.Structure):
    _fields_ = [("ndim", c_int32), ("n", c_int64 * 3), ("lo", c_double * 3), ("hi", c_double * 3),
                ("bc", c_int32 * 3), ("dtype", c_int32)]


class sc_linear_pde(ctypes.Structure):
    _fields_ = [("c", c_double * 3), ("nu_diff", c_double), ("beta", c_double), ("dt", c_double),
                ("order", c_int32), ("nn_policy", c_int32), ("nn_eps", c_double),
                ("block_len", c_double), ("split", c_int32), ("stages", c_int32)]


class sc_batch_item(ctypes.Structure):
    _fields_ = [("offset", c_int64), ("n", c_int64), ("nlines", c_int64), ("lo", c_double), ("hi", c_double),
                ("alpha", c_double), ("scale", c_double), ("g_offset", c_int64), ("bc", c_int32),
                ("op", c_int32), ("k", c_int32), ("axis", c_int32)]


class sc_hj_params(ctypes.Structure):
    _fields_ = [("beta", c_double), ("cfl", c_double), ("t_end", c_double), ("theta", c_double),
                ("weights", c_int32), ("hamiltonian", c_int32)]


HJ_WEIGHTS = {"linear": 0, "wenoz": 1, "learned": 2}
# "quadratic": u_t + (u_x^2 + u_y^2)/2 = 0; "ex3": Example 3, u_t + (1 + u_x + u_y)^2/2 = S (manufactured)
HJ_HAMILTONIANS = {"quadratic": 0, "ex3": 1}


@dataclass
class Grid:
    """Uniform grid: ``n[0]`` is the contiguous x axis."""
    n: Sequence[int]
    lo: Sequence[float] = field(default_factory=lambda: (0.0, 0.0, 0.0))
    hi: Sequence[float] = field(default_factory=lambda: (1.0, 1.0, 1.0))
    bc: Sequence[str] = field(default_factory=lambda: ("periodic",) * 3)
    dtype: int = SC_F64

    def c(self) -> sc_grid:
        g = sc_grid()
        nd = len(self.n)
        g.ndim = nd
        for e in range(3):
            g.n[e] = int(self.n[e]) if e < nd else 1
            g.lo[e] = float(self.lo[e]) if e < nd else 0.0
            g.hi[e] = float(self.hi[e]) if e < nd else 1.0
            g.bc[e] = BCS[self.bc[e]] if e < nd else 0
        g.dtype = self.dtype
        return g

    @property
    def shape(self):
        return tuple(int(x) for x in reversed(list(self.n)))

    def dx(self, dim: int) -> float:
        cells = self.n[dim] if self.bc[dim] == "periodic" else self.n[dim] - 1
        return (self.hi[dim] - self.lo[dim]) / cells


_lib = None


def load():
    """Load ``libsc.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2007_03041_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    gp = POINTER(sc_grid)
    lib.sc_local_quad.argtypes = [gp, c_int, c_int, c_double, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.sc_sweep_LR.argtypes = [gp, c_int, c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p]
    lib.sc_apply_invL.argtypes = [gp, c_int, c_int, c_int, c_double, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_size_t, c_void_p]
    lib.sc_apply_invL_noalloc.argtypes = [gp, c_int, c_int, c_int, c_double, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.sc_apply_invL_nn.argtypes = [gp, c_int, c_int, c_int, c_double, c_int64, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_size_t, c_void_p]
    lib.sc_chunk_points.argtypes = [gp, c_int]
    lib.sc_chunk_points.restype = c_int64
    lib.sc_apply_D_partial_sum.argtypes = [gp, c_int, c_int, c_int, c_double, c_int, c_double, c_void_p,
                                           c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    lib.sc_time_step.argtypes = [gp, POINTER(sc_linear_pde), c_int, c_void_p, c_void_p, c_size_t, c_void_p]
    lib.sc_workspace_bytes.argtypes = [gp, c_int, c_int, c_int]
    lib.sc_workspace_bytes.restype = c_size_t
    lib.sc_effective_dt.argtypes = [gp, POINTER(sc_linear_pde)]
    lib.sc_effective_dt.restype = c_double
    lib.sc_last_error.argtypes = []
    lib.sc_last_error.restype = c_char_p
    lib.sc_timing_enable.argtypes = [c_int]
    lib.sc_timing_select.argtypes = [ctypes.c_char_p]
    lib.sc_timing_read.argtypes = [POINTER(c_char * 64), POINTER(c_double), POINTER(c_int), c_int]
    lib.sc_timing_read.restype = c_int
    lib.sc_timing_reset.argtypes = []
    lib.sc_timing_reset.restype = None
    bp = c_void_p
    lib.sc_batch_plan_create.argtypes = [POINTER(sc_batch_item), c_int, c_int, c_int, POINTER(c_void_p)]
    lib.sc_batch_plan_destroy.argtypes = [bp]
    lib.sc_batch_workspace_bytes.argtypes = [bp]
    lib.sc_batch_workspace_bytes.restype = c_size_t
    lib.sc_batch_elements.argtypes = [bp]
    lib.sc_batch_elements.restype = c_int64
    lib.sc_batch_apply.argtypes = [bp, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_int, c_void_p]
    lib.sc_batch_apply_per_instance.argtypes = [bp, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    lib.sc_batch_tune.argtypes = [bp, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_int, c_void_p]
    lib.sc_batch_describe.argtypes = [bp, c_char_p, c_int]
    lib.sc_batch_describe.restype = c_int
    lib.sc_batch_tune_export.argtypes = [c_char_p, c_int]
    lib.sc_batch_tune_export.restype = c_int
    lib.sc_batch_tune_import.argtypes = [c_char_p]
    lib.sc_batch_tune_import.restype = c_int
    hp = POINTER(sc_hj_params)
    lib.sc_hj_workspace_bytes.argtypes = [gp]
    lib.sc_hj_workspace_bytes.restype = c_size_t
    lib.sc_hj_init.argtypes = [gp, hp, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    lib.sc_hj_step.argtypes = [gp, hp, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    lib.sc_hj_harvest.argtypes = [gp, hp, c_void_p, c_int, c_void_p, c_void_p, c_void_p]
    lib.sc_mlp_param_count.argtypes = []
    lib.sc_mlp_param_count.restype = c_int
    lib.sc_mlp_forward.argtypes = [c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
    lib.sc_mlp_grad_workspace_bytes.argtypes = [c_int64]
    lib.sc_mlp_grad_workspace_bytes.restype = c_size_t
    lib.sc_mlp_grad.argtypes = [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                c_void_p]
    lib.sc_mlp_adam.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int, ctypes.c_float, c_void_p]
    for f in ("sc_local_quad", "sc_sweep_LR", "sc_apply_invL", "sc_apply_invL_noalloc", "sc_apply_invL_nn",
              "sc_apply_D_partial_sum",
              "sc_time_step",
              "sc_timing_enable", "sc_timing_select", "sc_batch_plan_create", "sc_batch_plan_destroy", "sc_batch_apply",
              "sc_batch_apply_per_instance", "sc_batch_tune", "sc_hj_init", "sc_hj_step", "sc_hj_harvest",
              "sc_mlp_forward", "sc_mlp_grad", "sc_mlp_adam"):
        getattr(lib, f).restype = c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != SC_OK:
        raise ScError(status, load().sc_last_error().decode())


def _stream() -> int:
    import torch

    return torch.cuda.current_stream().cuda_stream


def _tensor_ok(t, grid: Grid, name: str):
    import torch

    want = torch.float64 if grid.dtype == SC_F64 else torch.float32
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != want:
        raise ValueError(f"{name} must be {want}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    n = 1
    for x in grid.n:
        n *= int(x)
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, grid has {n}")


def _workspace(nbytes: int, device):
    import torch

    if nbytes == 0:
        return None, 0
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


def _gptr(g, grid: Grid, dim: int):
    if g is None:
        return None
    import torch

    lines = 1
    for e, x in enumerate(grid.n):
        if e != dim:
            lines *= int(x)
    if not (g.is_cuda and g.dtype == torch.float64 and g.is_contiguous() and g.numel() == 2 * lines):
        raise ValueError("Dirichlet values: contiguous float64 device tensor with 2 values per line")
    return g.data_ptr()


def workspace_bytes(grid: Grid, dim: int, which: int, k: int = 1) -> int:
    gc = grid.c()
    return int(load().sc_workspace_bytes(ctypes.byref(gc), dim, which, k))


def local_quad(v, grid: Grid, dim: int, order: int, alpha: float):
    """(J_L, J_R) along ``dim``."""
    import torch

    lib = load()
    _tensor_ok(v, grid, "v")
    JL, JR = torch.empty_like(v), torch.empty_like(v)
    gc = grid.c()
    _check(lib.sc_local_quad(ctypes.byref(gc), dim, order, alpha, v.data_ptr(), JL.data_ptr(), JR.data_ptr(),
                             _stream()))
    return JL, JR


def sweep_LR(JL, JR, grid: Grid, dim: int, alpha: float):
    """(I_L, I_R, line_ends[lines, 2]) raw sweeps along ``dim``."""
    import torch

    lib = load()
    _tensor_ok(JL, grid, "JL")
    _tensor_ok(JR, grid, "JR")
    IL, IR = torch.empty_like(JL), torch.empty_like(JL)
    lines = JL.numel() // int(grid.n[dim])
    ends = torch.empty((lines, 2), dtype=torch.float64, device=JL.device)
    gc = grid.c()
    _check(lib.sc_sweep_LR(ctypes.byref(gc), dim, alpha, JL.data_ptr(), JR.data_ptr(), IL.data_ptr(),
                           IR.data_ptr(), ends.data_ptr(), _stream()))
    return IL, IR, ends


def apply_invL(v, grid: Grid, dim: int, op: str, order: int, alpha: float, g=None, out=None):
    """out = L_op^{-1}[v] along ``dim``."""
    import torch

    lib = load()
    _tensor_ok(v, grid, "v")
    out = torch.empty_like(v) if out is None else out
    _tensor_ok(out, grid, "out")
    gc = grid.c()
    ws, wsp = _workspace(int(lib.sc_workspace_bytes(ctypes.byref(gc), dim, 0, 0)), v.device)
    nbytes = 0 if ws is None else ws.numel() - 256
    _check(lib.sc_apply_invL(ctypes.byref(gc), dim, OPS[op], order, alpha, _gptr(g, grid, dim), v.data_ptr(),
                             out.data_ptr(), wsp, nbytes, _stream()))
    return out


def apply_invL_noalloc(v, grid: Grid, dim: int, op: str, order: int, alpha: float, g=None, out=None):
    """out = L_op^{-1}[v] along ``dim`` through ``sc_apply_invL_noalloc`` (no workspace: the
    library's fixed per-GPU scratch holds the chunk totals).  ``out`` must be given by callers that
    cannot allocate."""
    import torch

    lib = load()
    _tensor_ok(v, grid, "v")
    out = torch.empty_like(v) if out is None else out
    _tensor_ok(out, grid, "out")
    gc = grid.c()
    _check(lib.sc_apply_invL_noalloc(ctypes.byref(gc), dim, OPS[op], order, alpha, _gptr(g, grid, dim),
                                     v.data_ptr(), out.data_ptr(), _stream()))
    return out


def chunk_points(grid: Grid, dim: int) -> int:
    """Points per chunk of the passes along ``dim`` (virtual blocks are multiples of it)."""
    gc = grid.c()
    c = int(load().sc_chunk_points(ctypes.byref(gc), dim))
    if c < 0:
        raise ScError(SC_ERR_ARG, "invalid grid or dim")
    return c


def apply_invL_nn(v, grid: Grid, dim: int, op: str, order: int, alpha: float, block: int, g=None, out=None):
    """out = L_op^{-1}[v] along ``dim`` in the nearest-neighbour block form, virtual blocks of ``block``
    points (a multiple of chunk_points(grid, dim), or at least the line length)."""
    import torch

    lib = load()
    _tensor_ok(v, grid, "v")
    out = torch.empty_like(v) if out is None else out
    _tensor_ok(out, grid, "out")
    gc = grid.c()
    ws, wsp = _workspace(int(lib.sc_workspace_bytes(ctypes.byref(gc), dim, 0, 0)), v.device)
    nbytes = 0 if ws is None else ws.numel() - 256
    _check(lib.sc_apply_invL_nn(ctypes.byref(gc), dim, OPS[op], order, alpha, int(block), _gptr(g, grid, dim),
                                v.data_ptr(), out.data_ptr(), wsp, nbytes, _stream()))
    return out


def apply_D_partial_sum(v, grid: Grid, dim: int, op: str, order: int, alpha: float, k: int = 1,
                        scale: float = 1.0, g=None, out=None):
    """out = scale * sum_{p=1..k} D^p[v] along ``dim``."""
    import torch

    lib = load()
    _tensor_ok(v, grid, "v")
    out = torch.empty_like(v) if out is None else out
    _tensor_ok(out, grid, "out")
    gc = grid.c()
    ws, wsp = _workspace(int(lib.sc_workspace_bytes(ctypes.byref(gc), dim, 1, k)), v.device)
    nbytes = 0 if ws is None else ws.numel() - 256
    _check(lib.sc_apply_D_partial_sum(ctypes.byref(gc), dim, OPS[op], order, alpha, k, scale,
                                      _gptr(g, grid, dim), v.data_ptr(), out.data_ptr(), wsp, nbytes,
                                      _stream()))
    return out


def make_pde(c=(0.0, 0.0, 0.0), nu_diff=0.0, beta=1.0, dt=1e-3, order=6, nn_policy=0, nn_eps=0.0,
             block_len=0.0, split=False, stages=1) -> sc_linear_pde:
    p = sc_linear_pde()
    for e in range(3):
        p.c[e] = float(c[e]) if e < len(c) else 0.0
    p.nu_diff, p.beta, p.dt, p.order = float(nu_diff), float(beta), float(dt), int(order)
    p.nn_policy, p.nn_eps, p.block_len = int(nn_policy), float(nn_eps), float(block_len)
    p.split, p.stages = int(bool(split)), int(stages)
    return p


class TimeStepper:
    """Holds the workspace of repeated ``sc_time_step`` calls on one grid (allocated once)."""

    def __init__(self, grid: Grid, pde: sc_linear_pde, device="cuda"):
        self.grid, self.pde = grid, pde
        self._gc = grid.c()
        nbytes = int(load().sc_workspace_bytes(ctypes.byref(self._gc), 0, 2, max(1, int(pde.stages))))
        self._ws, self._wsp = _workspace(nbytes, device)
        self._nbytes = nbytes

    def step(self, u, nsteps: int = 1):
        _tensor_ok(u, self.grid, "u")
        _check(load().sc_time_step(ctypes.byref(self._gc), ctypes.byref(self.pde), nsteps, u.data_ptr(),
                                   self._wsp, self._nbytes, _stream()))
        return u


def time_step(u, grid: Grid, nsteps: int, c=(0.0, 0.0, 0.0), nu_diff=0.0, beta=1.0, dt=1e-3, order=6,
              nn_policy=0, nn_eps=0.0, block_len=0.0, split=False, stages=1):
    """Advance u (in place) by ``nsteps`` steps of u_t + c.grad u = nu_diff lap u: forward Euler with D
    (stages 1) or the s-stage Runge-Kutta form with partial sums S_s (stages 2, 3)."""
    pde = make_pde(c, nu_diff, beta, dt, order, nn_policy, nn_eps, block_len, split, stages)
    return TimeStepper(grid, pde, u.device).step(u, nsteps)


def effective_dt(grid: Grid, pde: sc_linear_pde) -> float:
    gc = grid.c()
    return float(load().sc_effective_dt(ctypes.byref(gc), ctypes.byref(pde)))


def timing_enable(on: bool = True):
    _check(load().sc_timing_enable(1 if on else 0))


def timing_select(names=None):
    """Time only the launches of these kernel names (None or empty: every launch)."""
    sel = ",".join(names) if names else ""
    _check(load().sc_timing_select(sel.encode() if sel else None))


def timing_reset():
    load().sc_timing_reset()


def timing_read(max_entries: int = 32):
    """{kernel name: (total ms, launches)} since the last reset (synchronises the events)."""
    lib = load()
    names = (c_char * 64 * max_entries)()
    ms = (c_double * max_entries)()
    cnt = (c_int * max_entries)()
    m = lib.sc_timing_read(ctypes.cast(names, POINTER(c_char * 64)), ms, cnt, max_entries)
    return {bytes(names[i]).split(b"\0", 1)[0].decode(): (ms[i], cnt[i]) for i in range(m)}


def batch_tune_save(path: str) -> int:
    """Writes the autotuner's table of this process to ``path`` (text); returns the classes saved."""
    lib = load()
    n = lib.sc_batch_tune_export(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib.sc_batch_tune_export(buf, n + 1)
    with open(path, "w") as f:
        f.write(buf.value.decode())
    return buf.value.count(b"\n")


def batch_tune_load(path: str) -> None:
    """Merges a table written by ``batch_tune_save`` into this process's autotuner table."""
    with open(path) as f:
        text = f.read()
    _check(load().sc_batch_tune_import(text.encode()))


class BatchPlan:
    """A plan over many independent instances (``sc_batch_*``).

    ``items``: sequence of dicts with keys offset, n, nlines, lo, hi, alpha, bc ("periodic" or
    "dirichlet"), op ("L", "R", "0"), k (0 or 1), and optionally scale (default 1), g_offset
    (default -1) and axis (default 0: contiguous lines; 1: interleaved lines, point p of line l at
    offset + p * nlines + l).  Arrays are flat contiguous device tensors of the plan's dtype (float64 for
    SC_F64, float32 for SC_F32_MIXED) with at least ``elements`` entries.
    """

    def __init__(self, items, dtype: int = SC_F64, order: int = 6, device="cuda"):
        lib = load()
        arr = (sc_batch_item * len(items))()
        for i, it in enumerate(items):
            e = arr[i]
            e.offset, e.n, e.nlines = int(it["offset"]), int(it["n"]), int(it["nlines"])
            e.lo, e.hi, e.alpha = float(it["lo"]), float(it["hi"]), float(it["alpha"])
            e.scale = float(it.get("scale", 1.0))
            e.g_offset = int(it.get("g_offset", -1))
            e.bc, e.op, e.k, e.axis = BCS[it["bc"]], OPS[it["op"]], int(it["k"]), int(it.get("axis", 0))
        self._h = c_void_p()
        _check(lib.sc_batch_plan_create(arr, len(items), dtype, order, ctypes.byref(self._h)))
        self.dtype, self.order, self.count = dtype, order, len(items)
        self.elements = int(lib.sc_batch_elements(self._h))
        self._ws, self._wsp = _workspace(int(lib.sc_batch_workspace_bytes(self._h)), device)
        self._nbytes = 0 if self._ws is None else self._ws.numel() - 256

    def _arrays(self, v, out, g):
        import torch

        want = torch.float64 if self.dtype == SC_F64 else torch.float32
        for name, t in (("v", v), ("out", out)):
            if not (t.is_cuda and t.dtype == want and t.is_contiguous() and t.numel() >= self.elements):
                raise ValueError(f"{name}: contiguous {want} device tensor with >= {self.elements} elements")
        if g is not None and not (g.is_cuda and g.dtype == torch.float64 and g.is_contiguous()):
            raise ValueError("g: contiguous float64 device tensor")
        return v.data_ptr(), out.data_ptr(), None if g is None else g.data_ptr()

    def apply(self, v, out=None, g=None, use_graph: bool = False):
        import torch

        out = torch.empty_like(v) if out is None else out
        vp, op_, gp = self._arrays(v, out, g)
        _check(load().sc_batch_apply(self._h, vp, op_, gp, self._wsp, self._nbytes, 1 if use_graph else 0,
                                     _stream()))
        return out

    def apply_per_instance(self, v, out=None, g=None):
        import torch

        out = torch.empty_like(v) if out is None else out
        vp, op_, gp = self._arrays(v, out, g)
        _check(load().sc_batch_apply_per_instance(self._h, vp, op_, gp, self._wsp, self._nbytes, _stream()))
        return out

    def tune(self, v, out=None, g=None, reps: int = 3):
        import torch

        out = torch.empty_like(v) if out is None else out
        vp, op_, gp = self._arrays(v, out, g)
        _check(load().sc_batch_tune(self._h, vp, op_, gp, self._wsp, self._nbytes, reps, _stream()))

    def describe(self) -> dict:
        import json

        lib = load()
        n = lib.sc_batch_describe(self._h, None, 0)
        buf = ctypes.create_string_buffer(n + 1)
        lib.sc_batch_describe(self._h, buf, n + 1)
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().sc_batch_plan_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------------
# Nonlinear Hamilton-Jacobi example and the learned weight proposer
# ------------------------------------------------------------------------------------------------
def _f32dev(t, name, shape_last=None):
    import torch

    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name}: contiguous float32 device tensor")
    if shape_last is not None and t.shape[-1] != shape_last:
        raise ValueError(f"{name}: last dimension must be {shape_last}")


class HJSolver:
    """u_t + H(u_x, u_y) = S on a periodic n x n grid of [0, L]^2 (``sc_hj_*``): ``hamiltonian``
    "quadratic" (|grad u|^2 / 2, S = 0) or "ex3" (Example 3 with its manufactured source); u is an
    (n1, n0) float64 device tensor updated in place."""

    def __init__(self, n, L=2 * 3.141592653589793, beta=1.0, cfl=1.0, t_end=1.0, weights="linear",
                 theta=0.05, device="cuda", hamiltonian="quadratic"):
        import torch

        n0, n1 = (n, n) if isinstance(n, int) else n
        self.grid = Grid((n0, n1), (0.0, 0.0), (L, L))
        self._gc = self.grid.c()
        self.p = sc_hj_params()
        self.p.beta, self.p.cfl, self.p.t_end, self.p.theta = beta, cfl, t_end, theta
        self.p.weights, self.p.hamiltonian = HJ_WEIGHTS[weights], HJ_HAMILTONIANS[hamiltonian]
        lib = load()
        nb = int(lib.sc_hj_workspace_bytes(ctypes.byref(self._gc)))
        if nb == 0:
            raise ScError(SC_ERR_ARG, "invalid grid")
        self._ws, self._wsp = _workspace(nb, device)
        self._nbytes = nb - 256
        self.state = torch.zeros(8, dtype=torch.float64, device=device)
        self.mlp = None

    def init(self, u):
        _tensor_ok(u, self.grid, "u")
        _check(load().sc_hj_init(ctypes.byref(self._gc), ctypes.byref(self.p), u.data_ptr(), self.state.data_ptr(),
                                 self._wsp, self._nbytes, _stream()))

    def step(self, u, nsteps=1):
        _tensor_ok(u, self.grid, "u")
        mp = None
        if self.p.weights == 2:
            if self.mlp is None:
                raise ValueError("learned weights: set .mlp to the proposer's parameters")
            _f32dev(self.mlp, "mlp")
            mp = self.mlp.data_ptr()
        _check(load().sc_hj_step(ctypes.byref(self._gc), ctypes.byref(self.p), nsteps, u.data_ptr(),
                                 self.state.data_ptr(), mp, self._wsp, self._nbytes, _stream()))
        return u

    def run_to(self, u, max_steps=100000, chunk=16):
        """Steps until the device-side time reaches t_end (checks every ``chunk`` steps)."""
        self.init(u)
        done = 0
        while done < max_steps:
            self.step(u, chunk)
            done += chunk
            if self.read_state()["t"] >= self.p.t_end - 1e-14:
                break
        return u

    def read_state(self):
        import torch

        torch.cuda.synchronize()
        s = self.state.cpu().tolist()
        return dict(c=s[0], t=s[1], steps=int(s[2]), fallbacks=s[3], judged_err_sum=s[4], judged=s[5])

    def harvest(self, u, axis):
        """(X, Y): features and WENO-Z weights of every stencil of u along ``axis`` (2 per point)."""
        import torch

        _tensor_ok(u, self.grid, "u")
        n = u.numel()
        X = torch.empty((2 * n, 8), dtype=torch.float32, device=u.device)
        Y = torch.empty((2 * n, 3), dtype=torch.float32, device=u.device)
        _check(load().sc_hj_harvest(ctypes.byref(self._gc), ctypes.byref(self.p), u.data_ptr(), axis, X.data_ptr(),
                                    Y.data_ptr(), _stream()))
        return X, Y


def mlp_param_count() -> int:
    return int(load().sc_mlp_param_count())


def mlp_forward(params, X):
    import torch

    _f32dev(params, "params")
    _f32dev(X, "X", 8)
    Y = torch.empty((X.shape[0], 3), dtype=torch.float32, device=X.device)
    _check(load().sc_mlp_forward(params.data_ptr(), X.shape[0], X.data_ptr(), Y.data_ptr(), _stream()))
    return Y


class MlpTrainer:
    """Gradient and Adam state of the proposer (all arithmetic in the library's kernels)."""

    def __init__(self, params, max_batch: int):
        import torch

        _f32dev(params, "params")
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.grad = torch.zeros_like(params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        nb = int(load().sc_mlp_grad_workspace_bytes(max_batch))
        self._ws = torch.empty(nb // 4 + 64, dtype=torch.float32, device=params.device)
        self._nbytes = nb
        self.max_batch = max_batch
        self.t = 0

    def gradient(self, X, Y):
        _f32dev(X, "X", 8)
        _f32dev(Y, "Y", 3)
        if X.shape[0] > self.max_batch:
            raise ValueError("batch larger than max_batch")
        _check(load().sc_mlp_grad(self.params.data_ptr(), X.shape[0], X.data_ptr(), Y.data_ptr(), self.grad.data_ptr(),
                                  self.loss.data_ptr(), self._ws.data_ptr(), self._nbytes, _stream()))
        return self.grad, self.loss

    def adam(self, lr: float):
        self.t += 1
        _check(load().sc_mlp_adam(self.params.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                  self.t, float(lr), _stream()))

    def step(self, X, Y, lr: float):
        self.gradient(X, Y)
        self.adam(lr)
        return self.loss
