"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by element.

Tolerances (FP64 path): L^{-1} and time-step results within 1e-12 * ||ref||_inf; D and its partial
sums within 1e-12 * ||v||_inf (D = v - L^{-1} v cancels by up to (alpha/k)^2, so the backward-stable
scale of its error is the operand's, not the result's).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2007_03041_amd import Grid, ScError
from paper_2007_03041_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-12
OPS = ("L", "R", "0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def ogrid(g: Grid):
    return oracle.make_grid(g.n, g.lo, g.hi, g.bc)


def err(got, ref, scale):
    return float(np.abs(got - ref).max() / max(scale, 1e-300))


# ------------------------------------------------------------------------------ config 1 (1-D)
@pytest.mark.parametrize("op", OPS)
def test_config1_line_invL_and_partial_sums(gpu_lib, op):
    sc = gpu_lib
    N = 1024
    v = W.noisy_sine_line(N, index=1)
    g = Grid((N,), (0.0,), (1.0,), ("periodic",))
    alpha = 1.0 / (1.0 * (1.0 / N))  # beta / (c dt), dt = dx
    ref = oracle.apply_invL(ogrid(g), 0, op, 6, alpha, v)
    got = host(sc.apply_invL(dev(v), g, 0, op, 6, alpha))
    assert err(got, ref, np.abs(ref).max()) < TOL
    for k in (1, 2, 3):
        ref = oracle.apply_D_partial_sum(ogrid(g), 0, op, 6, alpha, k, 1.0, v)
        got = host(sc.apply_D_partial_sum(dev(v), g, 0, op, 6, alpha, k, 1.0))
        assert err(got, ref, np.abs(v).max()) < TOL, k


def test_config1_replicated_lines(gpu_lib):
    sc = gpu_lib
    N, lines = 1024, 300
    v = W.noisy_sine_line(N, index=1, lines=lines)
    g = Grid((N, lines), (0.0, 0.0), (1.0, 1.0))
    for op in OPS:
        ref = oracle.apply_D_partial_sum(ogrid(g), 0, op, 6, 1024.0, 3, -1024.0 ** 2, v)
        got = host(sc.apply_D_partial_sum(dev(v), g, 0, op, 6, 1024.0, 3, -1024.0 ** 2))
        assert err(got, ref, 1024.0 ** 2 * np.abs(v).max()) < TOL


@pytest.mark.parametrize("k", [5, 8])
@pytest.mark.parametrize("dim", [0, 1])
def test_fused_high_powers_of_D(gpu_lib, k, dim):
    """S_k = D + ... + D^k fused in one pass for k up to 8 (whole periodic lines along x and y, each
    power's operand exchanged through the tile), every operator, against the oracle's powers."""
    sc = gpu_lib
    n = (256, 200)
    v = W.random_field((n[1], n[0]), index=40 + k + dim)
    g = Grid(n, (0.0, 0.0), (1.0, 0.8))
    alpha = 0.6 / g.dx(dim)
    for op in OPS:
        ref = oracle.apply_D_partial_sum(ogrid(g), dim, op, 6, alpha, k, -0.4, v)
        got = host(sc.apply_D_partial_sum(dev(v), g, dim, op, 6, alpha, k, -0.4))
        assert err(got, ref, max(np.abs(ref).max(), np.abs(v).max())) < TOL, op


# ------------------------------------------------------------------------------ ragged 1-D lines
CASES = []
_r = np.random.default_rng(5)
for n in (7, 9, 64, 100, 129, 256, 511, 512, 513, 1000, 1024, 2048, 2049, 4096, 4097, 9000, 16384):
    for bc in ("periodic", "dirichlet"):
        for order in (4, 6):
            CASES.append((n, bc, order, float(10 ** _r.uniform(-2, math.log10(20)))))


@pytest.mark.parametrize("n,bc,order,nu", CASES)
def test_ragged_lines_contiguous(gpu_lib, n, bc, order, nu):
    sc = gpu_lib
    lines = 3
    v = W.random_field((lines, n), index=20 + n)
    g = Grid((n, lines), (0.0, 0.0), (2.0, 1.0), (bc, "periodic"))
    alpha = nu / g.dx(0)
    gv = np.random.default_rng(n).standard_normal((lines, 2)) if bc == "dirichlet" else None
    for op in OPS:
        ref = oracle.apply_invL(ogrid(g), 0, op, order, alpha, v, gv)
        got = host(sc.apply_invL(dev(v), g, 0, op, order, alpha, g=None if gv is None else dev(gv)))
        assert err(got, ref, np.abs(ref).max()) < TOL, op
        ref = oracle.apply_D_partial_sum(ogrid(g), 0, op, order, alpha, 1, 1.0, v, gv)
        got = host(sc.apply_D_partial_sum(dev(v), g, 0, op, order, alpha, 1, 1.0,
                                          g=None if gv is None else dev(gv)))
        assert err(got, ref, np.abs(v).max()) < TOL, op
    if bc == "periodic":
        ref = oracle.apply_D_partial_sum(ogrid(g), 0, "0", order, alpha, 3, 1.0, v)
        got = host(sc.apply_D_partial_sum(dev(v), g, 0, "0", order, alpha, 3, 1.0))
        assert err(got, ref, np.abs(v).max()) < TOL


# ------------------------------------------------------------------------------ many long x lines
LONG_CASES = [(2049, "periodic", 4), (2049, "dirichlet", 6), (4096, "periodic", 6), (4096, "dirichlet", 4)]


@pytest.mark.parametrize("n,bc,order", LONG_CASES)
def test_many_long_x_lines(gpu_lib, n, bc, order):
    """One-line tiles (x lines of 1025..4096 points), more lines than the chip holds workgroups at
    once, ragged and full lengths, one and two operators per pass."""
    sc = gpu_lib
    lines = 700
    v = W.random_field((lines, n), index=60 + n)
    g = Grid((n, lines), (0.0, 0.0), (2.0, 1.0), (bc, "periodic"))
    alpha = 3.0 / g.dx(0)
    gv = np.random.default_rng(n + 1).standard_normal((lines, 2)) if bc == "dirichlet" else None
    for op in OPS:
        ref = oracle.apply_D_partial_sum(ogrid(g), 0, op, order, alpha, 1, 1.0, v, gv)
        got = host(sc.apply_D_partial_sum(dev(v), g, 0, op, order, alpha, 1, 1.0,
                                          g=None if gv is None else dev(gv)))
        assert err(got, ref, np.abs(v).max()) < TOL, op
    if bc == "periodic":
        # two operators on the same operand in one x pass (advection and diffusion of a time step)
        ref = oracle.time_step(ogrid(g), (0.7, -0.3), 0.05, 1.0, 0.5 / n, order, 1, v, split=True)
        u = dev(v)
        sc.time_step(u, g, 1, c=(0.7, -0.3), nu_diff=0.05, beta=1.0, dt=0.5 / n, order=order, split=True)
        assert err(host(u), ref, np.abs(ref).max()) < TOL


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_lines_of_many_chunks(gpu_lib, bc):
    """x lines of 18 chunks (ragged): the chunk carries come from their own launch, where lines of
    at most 16 chunks form them inside the apply launch."""
    sc = gpu_lib
    n, lines = 140000, 3
    v = W.random_field((lines, n), index=77)
    g = Grid((n, lines), (0.0, 0.0), (1.0, 1.0), (bc, "periodic"))
    alpha = 0.02 / g.dx(0)
    gv = np.random.default_rng(78).standard_normal((lines, 2)) if bc == "dirichlet" else None
    for op in OPS:
        ref = oracle.apply_D_partial_sum(ogrid(g), 0, op, 4, alpha, 1, 1.0, v, gv)
        got = host(sc.apply_D_partial_sum(dev(v), g, 0, op, 4, alpha, 1, 1.0, g=None if gv is None else dev(gv)))
        assert err(got, ref, np.abs(v).max()) < TOL, op


STRIDED_CHUNKED = [(4096, "periodic", 4), (4096, "dirichlet", 6), (4608, "dirichlet", 4), (4608, "periodic", 6),
                   (17408, "periodic", 4), (17408, "dirichlet", 6)]


@pytest.mark.parametrize("k", [2, 3, 5])
@pytest.mark.parametrize("n,dim", [(4096, 1), (20000, 0)])
def test_partial_sums_of_chunked_lines(gpu_lib, k, n, dim):
    """S_k on periodic lines longer than one tile (y lines of 8 chunks, x lines of 3): one chunked
    pass per power, every operator, against the oracle's powers."""
    sc = gpu_lib
    shape = (n, 5) if dim == 0 else (24, n)
    v = W.random_field(tuple(reversed(shape)), index=50 + k + dim)
    g = Grid(shape, (0.0, 0.0), (1.0, 1.0))
    alpha = 0.4 / g.dx(dim)
    for op in OPS:
        ref = oracle.apply_D_partial_sum(ogrid(g), dim, op, 6, alpha, k, -0.7, v)
        got = host(sc.apply_D_partial_sum(dev(v), g, dim, op, 6, alpha, k, -0.7))
        assert err(got, ref, max(np.abs(ref).max(), np.abs(v).max())) < TOL, op


@pytest.mark.parametrize("n,bc,order", STRIDED_CHUNKED)
def test_strided_chunked_full_lines(gpu_lib, n, bc, order):
    """y lines that are whole numbers of chunks: 8 chunks (carries formed in the apply launch from
    prefetched chunk totals), 9 chunks (from the totals read in the carry step) and 17 chunks (the
    carry launch), periodic and Dirichlet, against the oracle."""
    sc = gpu_lib
    cols = 16
    v = W.random_field((n, cols), index=90 + n)
    g = Grid((cols, n), (0.0, 0.0), (1.0, 3.0), ("periodic", bc))
    alpha = 0.05 / g.dx(1)
    gv = np.random.default_rng(n + 3).standard_normal((cols, 2)) if bc == "dirichlet" else None
    for op in OPS:
        ref = oracle.apply_D_partial_sum(ogrid(g), 1, op, order, alpha, 1, 1.0, v, gv)
        got = host(sc.apply_D_partial_sum(dev(v), g, 1, op, order, alpha, 1, 1.0, g=None if gv is None else dev(gv)))
        assert err(got, ref, np.abs(v).max()) < TOL, op
        ref = oracle.apply_invL(ogrid(g), 1, op, order, alpha, v, gv)
        got = host(sc.apply_invL(dev(v), g, 1, op, order, alpha, g=None if gv is None else dev(gv)))
        assert err(got, ref, np.abs(ref).max()) < TOL, op


# ------------------------------------------------------------------------------ strided axes
SHAPES = [
    ((41, 37, 5), ("periodic", "dirichlet", "periodic")),
    ((20, 1100, 3), ("periodic", "periodic", "periodic")),   # y lines longer than one tile
    ((17, 2, 600), ("dirichlet", "periodic", "dirichlet")),  # z lines longer than one tile
    ((33, 130, 9), ("dirichlet", "dirichlet", "periodic")),
]


@pytest.mark.parametrize("n,bcs", SHAPES)
def test_all_axes(gpu_lib, n, bcs):
    sc = gpu_lib
    shape = tuple(reversed(n))
    v = W.random_field(shape, index=40 + n[1])
    g = Grid(n, (0.0, -1.0, 0.5), (1.0, 2.0, 1.5), bcs)
    rng = np.random.default_rng(sum(n))
    for dim in range(3):
        if n[dim] < 7:
            continue
        alpha = float(rng.uniform(0.05, 5.0)) / g.dx(dim)
        lines = v.size // n[dim]
        gv = rng.standard_normal((lines, 2)) if bcs[dim] == "dirichlet" else None
        for order in (4, 6):
            for op in OPS:
                ref = oracle.apply_invL(ogrid(g), dim, op, order, alpha, v, gv)
                got = host(sc.apply_invL(dev(v), g, dim, op, order, alpha,
                                         g=None if gv is None else dev(gv)))
                assert err(got, ref, np.abs(ref).max()) < TOL, (dim, order, op)
        if bcs[dim] == "periodic":
            ref = oracle.apply_D_partial_sum(ogrid(g), dim, "R", 6, alpha, 2, alpha, v)
            got = host(sc.apply_D_partial_sum(dev(v), g, dim, "R", 6, alpha, 2, alpha))
            assert err(got, ref, alpha * np.abs(v).max()) < TOL, dim


# ------------------------------------------------------------------------------ stages
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_local_quad_and_sweeps(gpu_lib, bc):
    sc = gpu_lib
    n = (300, 7, 2)
    v = W.random_field(tuple(reversed(n)), index=77)
    g = Grid(n, (0, 0, 0), (1, 1, 1), (bc, bc, "periodic"))
    for dim, order in ((0, 6), (1, 4)):
        alpha = 0.7 / g.dx(dim)
        JLr, JRr = oracle.local_quad(ogrid(g), dim, order, alpha, v)
        JL, JR = sc.local_quad(dev(v), g, dim, order, alpha)
        assert err(host(JL), JLr, np.abs(JLr).max()) < TOL
        assert err(host(JR), JRr, np.abs(JRr).max()) < TOL
        ILr, IRr, ends_r = oracle.sweep_LR(ogrid(g), dim, alpha, JLr, JRr)
        IL, IR, ends = sc.sweep_LR(dev(JLr), dev(JRr), g, dim, alpha)
        assert err(host(IL), ILr, np.abs(ILr).max()) < TOL
        assert err(host(IR), IRr, np.abs(IRr).max()) < TOL
        assert err(host(ends), ends_r, np.abs(ends_r).max()) < TOL


# ------------------------------------------------------------------------------ time steps
def test_time_step_2d_advection_diffusion_small(gpu_lib):
    sc = gpu_lib
    N = 256
    u0 = W.fourier_field(N, N)
    g = Grid((N, N), (0, 0), (2 * np.pi, 2 * np.pi))
    dt = 2 * np.pi / N
    ref = oracle.time_step(ogrid(g), (1.0, 1.0), 1.0, 1.0, dt, 4, 3, u0)
    u = dev(u0)
    sc.time_step(u, g, 3, c=(1.0, 1.0), nu_diff=1.0, beta=1.0, dt=dt, order=4)
    assert err(host(u), ref, np.abs(ref).max()) < TOL


def test_time_step_mixed_signs_nonsquare(gpu_lib):
    sc = gpu_lib
    n = (96, 1030)  # y lines chunked
    u0 = W.random_field((n[1], n[0]), index=90)
    g = Grid(n, (0, 0), (1.0, 3.0))
    ref = oracle.time_step(ogrid(g), (-0.7, 0.4), 0.05, 1.0, 0.01, 6, 2, u0)
    u = dev(u0)
    sc.time_step(u, g, 2, c=(-0.7, 0.4), nu_diff=0.05, beta=1.0, dt=0.01, order=6)
    assert err(host(u), ref, np.abs(ref).max()) < TOL


@pytest.mark.parametrize("n", [(256, 256), (80, 1500)])
def test_time_step_split_form(gpu_lib, n):
    sc = gpu_lib
    u0 = W.random_field((n[1], n[0]), index=91)
    g = Grid(n, (0, 0), (2 * np.pi, 2 * np.pi))
    dt = 2 * np.pi / n[0]
    ref = oracle.time_step(ogrid(g), (1.0, 1.0), 1.0, 1.0, dt, 4, 3, u0, split=True)
    u = dev(u0)
    sc.time_step(u, g, 3, c=(1.0, 1.0), nu_diff=1.0, beta=1.0, dt=dt, order=4, split=True)
    assert err(host(u), ref, np.abs(ref).max()) < TOL


def test_time_step_3d_dirichlet_heat_split(gpu_lib):
    sc = gpu_lib
    n = 40
    u0 = W.bump_field(n)
    g = Grid((n, n, n), (0, 0, 0), (1, 1, 1), ("dirichlet",) * 3)
    dt = 1.0 / (n - 1)
    ref = oracle.time_step(ogrid(g), (0, 0, 0), 1.0, 1.0, dt, 6, 3, u0, split=True)
    u = dev(u0)
    sc.time_step(u, g, 3, nu_diff=1.0, beta=1.0, dt=dt, order=6, split=True)
    assert err(host(u), ref, np.abs(ref).max()) < TOL


@pytest.mark.parametrize("nsteps", [1, 2, 3])
def test_time_step_split_in_place_pass(gpu_lib, nsteps):
    """Dimension-split steps with an odd number of passes run the last pass whose lines fit one tile
    in place; here z lines are chunked (9000 points), so that pass is the y pass of the last step."""
    sc = gpu_lib
    n = (24, 20, 9000)
    u0 = W.random_field((n[2], n[1], n[0]), index=93)
    g = Grid(n, (0, 0, 0), (1.0, 1.0, 30.0))
    dt = 1.0 / 24
    ref = oracle.time_step(ogrid(g), (0.5, -1.0, 2.0), 0.2, 1.0, dt, 6, nsteps, u0, split=True)
    u = dev(u0)
    sc.time_step(u, g, nsteps, c=(0.5, -1.0, 2.0), nu_diff=0.2, beta=1.0, dt=dt, order=6, split=True)
    assert err(host(u), ref, np.abs(ref).max()) < TOL


def test_time_step_3d_dirichlet_heat(gpu_lib):
    sc = gpu_lib
    n = 33
    u0 = W.bump_field(n)
    g = Grid((n, n, n), (0, 0, 0), (1, 1, 1), ("dirichlet",) * 3)
    dt = 1.0 / (n - 1)
    ref = oracle.time_step(ogrid(g), (0, 0, 0), 1.0, 1.0, dt, 6, 2, u0)
    u = dev(u0)
    sc.time_step(u, g, 2, nu_diff=1.0, beta=1.0, dt=dt, order=6)
    assert err(host(u), ref, np.abs(ref).max()) < TOL


# ------------------------------------------------------------------------------ full sizes
def test_config2_full_size_one_step_sampled(gpu_lib):
    """4096^2, order 4, one step in the benchmark's launch configuration; sampled points are
    recomputed by the oracle from their own row and column."""
    sc = gpu_lib
    N = 4096
    L = 2 * np.pi
    dx = L / N
    g = Grid((N, N), (0, 0), (L, L))
    u = W.fourier_field(N, N, device="cuda")
    u0 = host(u).copy()
    sc.time_step(u, g, 1, c=(1.0, 1.0), nu_diff=1.0, beta=1.0, dt=dx, order=4)
    got = host(u)
    a_adv, a_dif = 1.0 / dx, 1.0 / math.sqrt(dx)
    rng = np.random.default_rng(4096)
    rows = rng.choice(N, 6, replace=False)
    cols = rng.choice(N, 6, replace=False)
    for j in rows:
        row = u0[j]
        dR = row - oracle.line_invL("periodic", "R", 4, a_adv, dx, row)
        d0 = row - oracle.line_invL("periodic", "0", 4, a_dif, dx, row)
        for i in cols:
            col = u0[:, i]
            eR = col - oracle.line_invL("periodic", "R", 4, a_adv, dx, col)
            e0 = col - oracle.line_invL("periodic", "0", 4, a_dif, dx, col)
            ref = u0[j, i] - dR[i] - d0[i] - eR[j] - e0[j]
            assert abs(got[j, i] - ref) < TOL * np.abs(u0).max()


def test_config2_full_field_split_steps(gpu_lib):
    """4096^2, order 4, two dimension-split steps exactly as the benchmark runs them (sc_time_step,
    split, one call per step): every element against the oracle's two split steps."""
    sc = gpu_lib
    N = 4096
    L = 2 * np.pi
    dx = L / N
    g = Grid((N, N), (0, 0), (L, L))
    u0 = W.fourier_field(N, N)
    ref = oracle.time_step(ogrid(g), (1.0, 1.0), 1.0, 1.0, dx, 4, 2, u0, split=True)
    u = dev(u0)
    pde = sc.make_pde(c=(1.0, 1.0), nu_diff=1.0, beta=1.0, dt=dx, order=4, split=True)
    st = sc.TimeStepper(g, pde)
    st.step(u, 1)
    st.step(u, 1)
    assert err(host(u), ref, np.abs(ref).max()) < TOL


def test_config2_ten_steps_match_mode_symbols(gpu_lib):
    """4096^2, order 4, 10 dimension-split steps (the benchmark's configuration): the 8-mode initial
    data evolves mode by mode, each multiplied per step by the product of the per-axis factors
    built from the discrete symbols (weights from the oracle)."""
    sc = gpu_lib
    N = 4096
    L = 2 * np.pi
    dx = L / N
    g = Grid((N, N), (0, 0), (L, L))
    u = W.fourier_field(N, N, device="cuda")
    sc.time_step(u, g, 10, c=(1.0, 1.0), nu_diff=1.0, beta=1.0, dt=dx, order=4, split=True)
    got = host(u)

    def sym(op, nu, th):
        mR, mL = list(range(-2, 2)), list(range(-1, 3))
        wR = oracle.weights(nu, [-m for m in mR])
        wL = oracle.weights(nu, mL)
        d = math.exp(-nu)
        sR = sum(w * np.exp(1j * th * m) for m, w in zip(mR, wR)) / (1 - d * np.exp(-1j * th))
        sL = sum(w * np.exp(1j * th * m) for m, w in zip(mL, wL)) / (1 - d * np.exp(1j * th))
        return sR if op == "R" else 0.5 * (sR + sL)

    a_adv, a_dif = 1.0 / dx, 1.0 / math.sqrt(dx)
    ks, amp, phase = W.fourier_modes(index=2)
    rng = np.random.default_rng(10)
    js, is_ = rng.choice(N, 64), rng.choice(N, 64)
    x, y = is_ * dx, js * dx
    ref = np.zeros(64)
    for (kx, ky), a, ph in zip(ks, amp, phase):
        S = 1.0
        for k in (kx, ky):
            th = k * dx
            S *= 1 - (1 - sym("R", a_adv * dx, th)) - (1 - sym("0", a_dif * dx, th))
        ref += np.real(a * np.exp(1j * ph) * S ** 10 * np.exp(1j * (kx * x + ky * y)))
    assert np.abs(got[js, is_] - ref).max() < TOL * np.abs(ref).max()


def test_config3_full_size_one_step_sampled(gpu_lib):
    """512^3 Dirichlet heat, order 6, one step; sampled points from their x, y and z lines."""
    sc = gpu_lib
    n = 512
    dx = 1.0 / (n - 1)
    g = Grid((n, n, n), (0, 0, 0), (1, 1, 1), ("dirichlet",) * 3)
    u = W.bump_field(n, device="cuda")
    u0 = host(u).copy()
    sc.time_step(u, g, 1, nu_diff=1.0, beta=1.0, dt=dx, order=6)
    got = host(u)
    a = 1.0 / math.sqrt(dx)
    rng = np.random.default_rng(512)
    for _ in range(12):
        k, j, i = rng.integers(0, n, 3)
        ref = u0[k, j, i]
        for line, pos in ((u0[k, j, :], i), (u0[k, :, i], j), (u0[:, j, i], k)):
            ref -= line[pos] - oracle.line_invL("dirichlet", "0", 6, a, dx, line)[pos]
        assert abs(got[k, j, i] - ref) < TOL * np.abs(u0).max()


# ------------------------------------------------------------------------------ errors
def test_invalid_arguments_raise(gpu_lib):
    sc = gpu_lib
    v = dev(np.ones(64))
    g = Grid((64,))
    with pytest.raises(ScError):
        sc.apply_invL(v, g, 0, "0", 5, 10.0)       # bad order
    with pytest.raises(ScError):
        sc.apply_invL(v, g, 0, "0", 6, -1.0)       # alpha <= 0
    with pytest.raises(ScError):
        sc.apply_invL(v, g, 1, "0", 6, 10.0)       # bad dim
    with pytest.raises(ScError):
        sc.apply_D_partial_sum(v, g, 0, "0", 6, 10.0, k=9)
    with pytest.raises(ScError):
        sc.apply_invL(dev(np.ones(6)), Grid((6,)), 0, "0", 6, 10.0)  # too short
    with pytest.raises(ScError):
        sc.apply_invL(v, g, 0, "0", 6, 10.0, out=v)  # aliasing
    gd = Grid((64,), bc=("dirichlet",))
    with pytest.raises(ScError):
        sc.apply_D_partial_sum(v, gd, 0, "0", 6, 10.0, k=2)  # unsupported


def test_nonfinite_input_propagates(gpu_lib):
    sc = gpu_lib
    a = np.ones(100)
    a[50] = np.nan
    out = host(sc.apply_invL(dev(a), Grid((100,)), 0, "0", 6, 100.0))
    assert np.isnan(out).any()


def test_repeat_runs_bitwise_identical(gpu_lib):
    """No LDS race: the same launch twice gives identical bits."""
    sc = gpu_lib
    n = (4096, 64)
    v = dev(W.random_field((64, 4096), index=3))
    g = Grid(n)
    a = host(sc.apply_D_partial_sum(v, g, 0, "0", 6, 900.0, 3, 1.0)).copy()
    b = host(sc.apply_D_partial_sum(v, g, 0, "0", 6, 900.0, 3, 1.0))
    assert np.array_equal(a, b)
    a = host(sc.apply_invL(v, g, 1, "R", 4, 30.0)).copy()
    b = host(sc.apply_invL(v, g, 1, "R", 4, 30.0))
    assert np.array_equal(a, b)


def test_timing_select_times_only_the_named_kernels(gpu_lib):
    """sc_timing_select: with a selection only the named launches carry events; without one every
    launch of the library does."""
    sc = gpu_lib
    n = (2048, 64)
    g = Grid(n)
    u = dev(W.random_field((64, 2048), index=5))
    try:
        sc.timing_reset()
        sc.timing_select(["line_pass_fused_y"])
        sc.timing_enable(True)
        sc.time_step(u, g, 2, c=(1.0, 1.0), nu_diff=0.5, beta=1.0, dt=1.0 / 2048, order=4, split=True)
        torch.cuda.synchronize()
        sc.timing_enable(False)
        sel = sc.timing_read()
        sc.timing_reset()
        sc.timing_select(None)
        sc.timing_enable(True)
        sc.time_step(u, g, 2, c=(1.0, 1.0), nu_diff=0.5, beta=1.0, dt=1.0 / 2048, order=4, split=True)
        torch.cuda.synchronize()
        sc.timing_enable(False)
        every = sc.timing_read()
    finally:
        sc.timing_enable(False)
        sc.timing_reset()
        sc.timing_select(None)
    assert set(sel) == {"line_pass_fused_y"} and sel["line_pass_fused_y"][1] == 2
    assert {"line_pass_fused_x", "line_pass_fused_y"} <= set(every)
    assert all(cnt == 2 and ms > 0 for ms, cnt in every.values())


# ------------------------------------------------------------------------------ pipelined strided passes
PIPE_CASES = [
    # (grid n (x, y, z), dim, bc, order): y and z lines of exactly one 512-point tile, enough line
    # tiles that workgroups of the persistent launch take several
    ((64, 512, 160), 1, "periodic", 6),
    ((64, 160, 512), 2, "dirichlet", 4),
    ((64, 512, 160), 1, "dirichlet", 6),
    ((32, 96, 512), 2, "periodic", 4),
]


@pytest.mark.parametrize("n,dim,bc,order", PIPE_CASES)
def test_pipelined_strided_whole_line_passes(gpu_lib, n, dim, bc, order, monkeypatch):
    """Strided passes whose lines fill one tile run persistent, their tiles loaded straight into LDS
    while the previous tile is finished (SC_PIPE=1: wherever the shape allows, not only where it
    is the faster form): every operator against the oracle, with Dirichlet values."""
    sc = gpu_lib
    monkeypatch.setenv("SC_PIPE", "1")
    v = W.random_field((n[2], n[1], n[0]), index=97 + dim)
    g = Grid(n, (0.0, 0.0, 0.0), (1.0, 2.0, 3.0), (bc, bc, bc))
    alpha = 0.07 / g.dx(dim)
    lines = v.size // n[dim]
    gv = np.random.default_rng(7).uniform(-1, 1, (lines, 2)) if bc == "dirichlet" else None
    for op in OPS:
        ref = oracle.apply_invL(ogrid(g), dim, op, order, alpha, v, gv)
        got = host(sc.apply_invL(dev(v), g, dim, op, order, alpha, g=None if gv is None else dev(gv)))
        assert err(got, ref, np.abs(ref).max()) < TOL, op
    ref = oracle.apply_D_partial_sum(ogrid(g), dim, "0", order, alpha, 1, -2.5, v, gv)
    got = host(sc.apply_D_partial_sum(dev(v), g, dim, "0", order, alpha, 1, -2.5, g=None if gv is None else dev(gv)))
    assert err(got, ref, 2.5 * np.abs(v).max()) < TOL


@pytest.mark.parametrize("pipe", ["1", ""])
def test_pipelined_passes_two_operators_in_a_time_step(gpu_lib, pipe, monkeypatch):
    """Advection and diffusion in one pass (two operators) on 512-point y and z lines, split steps
    with the last pass in place; the pipelined form forced, and the default choice."""
    sc = gpu_lib
    if pipe:
        monkeypatch.setenv("SC_PIPE", pipe)
    n = (48, 512, 512)
    u0 = W.random_field((n[2], n[1], n[0]), index=99)
    g = Grid(n, (0, 0, 0), (1.0, 4.0, 4.0))
    dt = 1.0 / 48
    ref = oracle.time_step(ogrid(g), (0.5, 1.0, -1.5), 0.1, 1.0, dt, 6, 1, u0, split=True)
    u = dev(u0)
    sc.time_step(u, g, 1, c=(0.5, 1.0, -1.5), nu_diff=0.1, beta=1.0, dt=dt, order=6, split=True)
    assert err(host(u), ref, np.abs(ref).max()) < TOL


def test_pipelined_and_tiled_passes_agree_bitwise(gpu_lib, monkeypatch):
    """The pipelined form computes exactly what the tile-per-workgroup form computes (same
    operations per point): SC_PIPE=0 selects the latter."""
    sc = gpu_lib
    n = (64, 512, 40)
    v = dev(W.random_field((n[2], n[1], n[0]), index=98))
    g = Grid(n, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), ("dirichlet",) * 3)
    monkeypatch.setenv("SC_PIPE", "1")
    a = host(sc.apply_invL(v, g, 1, "0", 6, 30.0)).copy()
    monkeypatch.setenv("SC_PIPE", "0")
    b = host(sc.apply_invL(v, g, 1, "0", 6, 30.0))
    assert np.array_equal(a, b)


# ------------------------------------------------------------------------------ single-pass chunked lines
SINGLE_CASES = [
    ((256, 4096), 1, "periodic", 4),     # y lines of 8 chunks (the 4096^2 workload's y pass, fewer lines)
    ((20000, 6), 0, "dirichlet", 6),     # x lines of 3 chunks, ragged
    ((48, 2200, 3), 1, "dirichlet", 6),  # y lines of 5 chunks, ragged
    ((40, 3, 1700), 2, "periodic", 4),   # z lines of 4 chunks, ragged
]


@pytest.mark.parametrize("n,dim,bc,order", SINGLE_CASES)
def test_single_pass_chunked_lines(gpu_lib, n, dim, bc, order, monkeypatch):
    """Lines of 2..8 chunks in one launch (SC_SINGLE=1: each tile publishes its chunk totals and
    gathers the others'): against the oracle, and bit for bit against the aggregate + apply launches."""
    sc = gpu_lib
    v = W.random_field(tuple(reversed(n)), index=71 + dim)
    g = Grid(n, tuple(0.0 for _ in n), tuple(1.0 + e for e in range(len(n))), tuple(bc for _ in n))
    lines = v.size // n[dim]
    gv = np.random.default_rng(3).uniform(-1, 1, (lines, 2)) if bc == "dirichlet" else None
    for op, nu in (("0", 0.03), ("R", 1.0), ("L", 0.2)):
        alpha = nu / g.dx(dim)
        ref = oracle.apply_invL(ogrid(g), dim, op, order, alpha, v, gv)
        monkeypatch.setenv("SC_SINGLE", "1")
        got = host(sc.apply_invL(dev(v), g, dim, op, order, alpha, g=None if gv is None else dev(gv))).copy()
        monkeypatch.delenv("SC_SINGLE")
        assert err(got, ref, np.abs(ref).max()) < TOL, op
        two = host(sc.apply_invL(dev(v), g, dim, op, order, alpha, g=None if gv is None else dev(gv)))
        assert np.array_equal(got, two), op


def test_single_pass_bounded_wait_gives_up_with_nan(gpu_lib, monkeypatch):
    """The gather's wait is bounded: forced from the host to give up (SC_SPIN_LIMIT=-m: published
    totals are ignored, m polls), every tile of a chunked line writes NaN and the launch ends; the
    next call, with the default limit, is correct again."""
    sc = gpu_lib
    n = (128, 4096)
    v = W.random_field((n[1], n[0]), index=72)
    g = Grid(n)
    monkeypatch.setenv("SC_SINGLE", "1")
    monkeypatch.setenv("SC_SPIN_LIMIT", "-3")
    out = host(sc.apply_invL(dev(v), g, 1, "0", 4, 40.0))
    assert np.isnan(out).all()
    monkeypatch.delenv("SC_SPIN_LIMIT")
    ref = oracle.apply_invL(ogrid(g), 1, "0", 4, 40.0, v)
    got = host(sc.apply_invL(dev(v), g, 1, "0", 4, 40.0))
    assert err(got, ref, np.abs(ref).max()) < TOL


# ------------------------------------------------------------------------------ windowed chunk carries
WINDOW_CASES = [
    (3 * 8192 + 500, "periodic", 1.0),
    (3 * 8192 + 500, "dirichlet", 1.0),
    (2 * 8192 + 200, "periodic", 0.4),   # K = 104
    (2 * 8192 + 200, "dirichlet", 0.4),
    (40000, "periodic", 2.0),
    (40000, "dirichlet", 0.33),          # K = 127
]


@pytest.mark.parametrize("n,bc,nu", WINDOW_CASES)
def test_windowed_chunk_carries(gpu_lib, n, bc, nu, monkeypatch):
    """Chunked x lines whose decay over K = ceil(60 ln 2 / nu) <= 128 points is below 2^-60: one apply
    launch whose carries are the sweeps over the K points beyond each chunk.  Against the oracle
    (1e-12) and against the exact aggregate + apply launches (SC_WINDOW=0) to 1e-15 of the result."""
    sc = gpu_lib
    lines = 3
    v = W.random_field((lines, n), index=90 + n % 97)
    g = Grid((n, lines), (0.0, 0.0), (1.0, 1.0), (bc, "periodic"))
    gv = np.random.default_rng(4).uniform(-1, 1, (lines, 2)) if bc == "dirichlet" else None
    alpha = nu / g.dx(0)
    for op in OPS:
        ref = oracle.apply_invL(ogrid(g), 0, op, 6, alpha, v, gv)
        sc.timing_reset()
        sc.timing_select(None)
        sc.timing_enable(True)
        got = host(sc.apply_invL(dev(v), g, 0, op, 6, alpha, g=None if gv is None else dev(gv)))
        sc.timing_enable(False)
        names = set(sc.timing_read())
        assert names == {"line_pass_apply_x"}, names  # the windowed form ran: no aggregate launch
        assert err(got, ref, np.abs(ref).max()) < TOL, op
        monkeypatch.setenv("SC_WINDOW", "0")
        exact = host(sc.apply_invL(dev(v), g, 0, op, 6, alpha, g=None if gv is None else dev(gv)))
        monkeypatch.delenv("SC_WINDOW")
        assert err(got, exact, np.abs(exact).max()) < 1e-15 * 8, op
        refd = oracle.apply_D_partial_sum(ogrid(g), 0, op, 6, alpha, 1, 1.0, v, gv)
        gotd = host(sc.apply_D_partial_sum(dev(v), g, 0, op, 6, alpha, 1, 1.0, g=None if gv is None else dev(gv)))
        assert err(gotd, refd, np.abs(v).max()) < TOL, op


def test_windowed_carries_not_taken_when_the_window_is_long(gpu_lib):
    """nu = 0.2 (K = 208 > 128), or a last chunk shorter than K: the exact aggregate + apply launches."""
    sc = gpu_lib
    for n, nu in ((3 * 8192 + 500, 0.2), (2 * 8192 + 40, 1.0)):
        v = W.random_field((2, n), index=91)
        g = Grid((n, 2), (0.0, 0.0), (1.0, 1.0))
        alpha = nu / g.dx(0)
        sc.timing_reset()
        sc.timing_select(None)
        sc.timing_enable(True)
        got = host(sc.apply_invL(dev(v), g, 0, "0", 6, alpha))
        sc.timing_enable(False)
        assert "line_pass_agg_x" in set(sc.timing_read()), n
        ref = oracle.apply_invL(ogrid(g), 0, "0", 6, alpha, v)
        assert err(got, ref, np.abs(ref).max()) < TOL
