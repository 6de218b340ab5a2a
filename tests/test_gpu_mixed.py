"""GPU parity of the mixed-precision path (SC_F32_MIXED) against the FP64 oracle.

The mixed path stores the operand and result in FP32 and computes the local integrals, segment
totals and re-sweeps in FP32; the in-wave scan of the segment totals is compensated (hi/lo float
pairs), and the carries across wave-parts and chunks and the boundary constants are FP64.  The GPU
receives the FP32 rounding of the oracle's FP64 input, so every error below includes that rounding.

Tolerance 1e-5, normalised as for the FP64 path: L^{-1} and time-step results relative to
||ref||_inf, D and its partial sums relative to |scale| ||v||_inf.
"""
import dataclasses
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2007_03041_amd import SC_F32_MIXED, Grid
from paper_2007_03041_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5
OPS = ("L", "R", "0")


def mixed(g: Grid) -> Grid:
    return dataclasses.replace(g, dtype=SC_F32_MIXED)


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def ogrid(g: Grid):
    return oracle.make_grid(g.n, g.lo, g.hi, g.bc)


def err(got, ref, scale):
    return float(np.abs(got - ref).max() / max(scale, 1e-300))


def test_config1_line_mixed(gpu_lib):
    sc = gpu_lib
    N = 1024
    v = W.noisy_sine_line(N, index=1)
    g = Grid((N,), (0.0,), (1.0,), ("periodic",))
    alpha = float(N)
    for op in OPS:
        ref = oracle.apply_invL(ogrid(g), 0, op, 6, alpha, v)
        got = host(sc.apply_invL(dev32(v), mixed(g), 0, op, 6, alpha))
        assert err(got, ref, np.abs(ref).max()) < TOL, op
        for k in (1, 2, 3):
            ref = oracle.apply_D_partial_sum(ogrid(g), 0, op, 6, alpha, k, -alpha ** 2, v)
            got = host(sc.apply_D_partial_sum(dev32(v), mixed(g), 0, op, 6, alpha, k, -alpha ** 2))
            assert err(got, ref, alpha ** 2 * np.abs(v).max()) < TOL, (op, k)


CASES = []
_r = np.random.default_rng(15)
for n in (7, 100, 513, 2049, 4097, 9000):
    for bc in ("periodic", "dirichlet"):
        for order in (4, 6):
            CASES.append((n, bc, order, float(10 ** _r.uniform(-3, math.log10(20)))))


@pytest.mark.parametrize("n,bc,order,nu", CASES)
def test_ragged_lines_mixed(gpu_lib, n, bc, order, nu):
    sc = gpu_lib
    lines = 5
    v = W.random_field((lines, n), index=120 + n)
    g = Grid((n, lines), (0.0, 0.0), (2.0, 1.0), (bc, "periodic"))
    alpha = nu / g.dx(0)
    gv = np.random.default_rng(n).standard_normal((lines, 2)) if bc == "dirichlet" else None
    for op in OPS:
        ref = oracle.apply_invL(ogrid(g), 0, op, order, alpha, v, gv)
        got = host(sc.apply_invL(dev32(v), mixed(g), 0, op, order, alpha, g=None if gv is None else dev64(gv)))
        assert err(got, ref, np.abs(ref).max()) < TOL, op
        ref = oracle.apply_D_partial_sum(ogrid(g), 0, op, order, alpha, 1, 1.0, v, gv)
        got = host(sc.apply_D_partial_sum(dev32(v), mixed(g), 0, op, order, alpha, 1, 1.0,
                                          g=None if gv is None else dev64(gv)))
        assert err(got, ref, np.abs(v).max()) < TOL, op
    if bc == "periodic":
        ref = oracle.apply_D_partial_sum(ogrid(g), 0, "0", order, alpha, 3, 1.0, v)
        got = host(sc.apply_D_partial_sum(dev32(v), mixed(g), 0, "0", order, alpha, 3, 1.0))
        assert err(got, ref, np.abs(v).max()) < TOL


SHAPES = [
    ((41, 37, 5), ("periodic", "dirichlet", "periodic")),
    ((20, 1100, 3), ("periodic", "periodic", "periodic")),   # y lines longer than one tile
    ((17, 2, 600), ("dirichlet", "periodic", "dirichlet")),  # z lines longer than one tile
    ((33, 130, 40), ("dirichlet", "dirichlet", "periodic")),
]


@pytest.mark.parametrize("n,bcs", SHAPES)
def test_all_axes_mixed(gpu_lib, n, bcs):
    sc = gpu_lib
    v = W.random_field(tuple(reversed(n)), index=140 + n[1])
    g = Grid(n, (0.0, -1.0, 0.5), (1.0, 2.0, 1.5), bcs)
    rng = np.random.default_rng(sum(n) + 1)
    for dim in range(3):
        if n[dim] < 7:
            continue
        alpha = float(rng.uniform(0.01, 5.0)) / g.dx(dim)
        lines = v.size // n[dim]
        gv = rng.standard_normal((lines, 2)) if bcs[dim] == "dirichlet" else None
        for order in (4, 6):
            for op in OPS:
                ref = oracle.apply_invL(ogrid(g), dim, op, order, alpha, v, gv)
                got = host(sc.apply_invL(dev32(v), mixed(g), dim, op, order, alpha,
                                         g=None if gv is None else dev64(gv)))
                assert err(got, ref, np.abs(ref).max()) < TOL, (dim, order, op)
        if bcs[dim] == "periodic":
            ref = oracle.apply_D_partial_sum(ogrid(g), dim, "R", 6, alpha, 2, alpha, v)
            got = host(sc.apply_D_partial_sum(dev32(v), mixed(g), dim, "R", 6, alpha, 2, alpha))
            assert err(got, ref, alpha * np.abs(v).max()) < TOL, dim


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_local_quad_and_sweeps_mixed(gpu_lib, bc):
    sc = gpu_lib
    n = (300, 7, 2)
    v = W.random_field(tuple(reversed(n)), index=177)
    g = Grid(n, (0, 0, 0), (1, 1, 1), (bc, bc, "periodic"))
    for dim, order in ((0, 6), (1, 4)):
        alpha = 0.7 / g.dx(dim)
        JLr, JRr = oracle.local_quad(ogrid(g), dim, order, alpha, v)
        JL, JR = sc.local_quad(dev32(v), mixed(g), dim, order, alpha)
        assert err(host(JL), JLr, np.abs(JLr).max()) < TOL
        assert err(host(JR), JRr, np.abs(JRr).max()) < TOL
        ILr, IRr, ends_r = oracle.sweep_LR(ogrid(g), dim, alpha, JLr, JRr)
        IL, IR, ends = sc.sweep_LR(dev32(JLr), dev32(JRr), mixed(g), dim, alpha)
        assert err(host(IL), ILr, np.abs(ILr).max()) < TOL
        assert err(host(IR), IRr, np.abs(IRr).max()) < TOL
        assert err(host(ends), ends_r, np.abs(ends_r).max()) < TOL


@pytest.mark.parametrize("split,steps", [(False, 1), (True, 3)])
def test_time_step_2d_mixed(gpu_lib, split, steps):
    """Unsplit steps at beta = 1 multiply grid-scale modes by |1 - d(beta + beta^2)| = 3 in 2-D, so
    rounding noise of any precision grows 3x per step; the unsplit form is checked over one step,
    the split form (every factor of modulus <= 1) over three."""
    sc = gpu_lib
    n = (256, 1030)  # y lines chunked
    u0 = W.fourier_field(*n)
    g = Grid(n, (0, 0), (2 * np.pi, 2 * np.pi * n[1] / n[0]))
    dt = 2 * np.pi / n[0]
    ref = oracle.time_step(ogrid(g), (1.0, 1.0), 1.0, 1.0, dt, 4, steps, u0, split=split)
    u = dev32(u0)
    sc.time_step(u, mixed(g), steps, c=(1.0, 1.0), nu_diff=1.0, beta=1.0, dt=dt, order=4, split=split)
    assert err(host(u), ref, np.abs(ref).max()) < TOL


def test_config3_full_size_five_steps_mixed_and_fp64(gpu_lib):
    """512^3 Dirichlet heat, order 6, 5 dimension-split steps (the unsplit beta = 1 step doubles
    grid-scale modes in 3-D): the mixed path and the FP64 path on the GPU against the oracle's 5
    steps over the whole field."""
    sc = gpu_lib
    n, steps = 512, 5
    dx = 1.0 / (n - 1)
    g = Grid((n, n, n), (0, 0, 0), (1, 1, 1), ("dirichlet",) * 3)
    u0 = W.bump_field(n)
    ref = oracle.time_step(ogrid(g), (0, 0, 0), 1.0, 1.0, dx, 6, steps, u0, split=True)
    scale = np.abs(ref).max()
    u = dev64(u0)
    sc.time_step(u, g, steps, nu_diff=1.0, beta=1.0, dt=dx, order=6, split=True)
    e64 = err(host(u), ref, scale)
    del u
    u = dev32(u0)
    sc.time_step(u, mixed(g), steps, nu_diff=1.0, beta=1.0, dt=dx, order=6, split=True)
    e32 = err(host(u), ref, scale)
    print(f"config 3, 5 steps: FP64 path err {e64:.3e}, mixed path err {e32:.3e}")
    assert e64 < 1e-12
    assert e32 < TOL


def test_repeat_runs_bitwise_identical_mixed(gpu_lib):
    sc = gpu_lib
    v = dev32(W.random_field((64, 4096), index=3))
    g = mixed(Grid((4096, 64)))
    a = host(sc.apply_D_partial_sum(v, g, 0, "0", 6, 900.0, 3, 1.0)).copy()
    b = host(sc.apply_D_partial_sum(v, g, 0, "0", 6, 900.0, 3, 1.0))
    assert np.array_equal(a, b)
    a = host(sc.apply_invL(v, g, 1, "R", 4, 30.0)).copy()
    b = host(sc.apply_invL(v, g, 1, "R", 4, 30.0))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n,dim,bc", [((64, 512, 160), 1, "dirichlet"), ((64, 160, 512), 2, "periodic")])
def test_pipelined_strided_passes_mixed(gpu_lib, n, dim, bc):
    """FP32 y/z lines of one 512-point tile: the persistent pipelined form (32 lines a tile, loaded
    straight into LDS), more line tiles than resident workgroups."""
    sc = gpu_lib
    v = W.random_field((n[2], n[1], n[0]), index=150 + dim)
    g = Grid(n, (0.0, 0.0, 0.0), (1.0, 2.0, 3.0), (bc, bc, bc))
    alpha = 0.05 / g.dx(dim)
    lines = v.size // n[dim]
    gv = np.random.default_rng(8).uniform(-1, 1, (lines, 2)) if bc == "dirichlet" else None
    for op in OPS:
        ref = oracle.apply_invL(ogrid(g), dim, op, 6, alpha, v, gv)
        got = host(sc.apply_invL(dev32(v), mixed(g), dim, op, 6, alpha, g=None if gv is None else dev64(gv)))
        assert err(got, ref, np.abs(ref).max()) < TOL, op


@pytest.mark.parametrize("mu", [0.95, 0.6, 0.45, 0.2, 1e-3])
def test_dirichlet_L0_end_constants_mixed(gpu_lib, mu):
    """L_0^{-1} on Dirichlet lines with random end values, alpha (b - a) = -ln mu: for mu near 1 the
    2x2 end-value constants exceed the result and cancel in it (they are summed per point in FP64);
    for mu <= 1/2 they ride through the FP32 sweeps.  Both within 1e-5 of the oracle, along x, y, z."""
    sc = gpu_lib
    n = (300, 40, 33)
    v = W.random_field((n[2], n[1], n[0]), index=160)
    g = Grid(n, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), ("dirichlet",) * 3)
    for dim in range(3):
        alpha = -math.log(mu)  # (b - a) = 1
        lines = v.size // n[dim]
        gv = np.random.default_rng(dim).uniform(-1, 1, (lines, 2))
        ref = oracle.apply_invL(ogrid(g), dim, "0", 6, alpha, v, gv)
        got = host(sc.apply_invL(dev32(v), mixed(g), dim, "0", 6, alpha, g=dev64(gv)))
        assert err(got, ref, np.abs(ref).max()) < TOL, dim
