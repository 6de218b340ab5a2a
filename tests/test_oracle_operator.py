"""Pins of the oracle's L^{-1}, D and partial sums against things outside the oracle (CPU only).

  * brute-force O(N^2) sums of the local integrals (periodic images summed in closed form);
  * direct mpmath integration of the periodic Green's function against the piecewise interpolant
    (never touches the recurrences or the weights);
  * discrete Fourier symbols applied with numpy's FFT;
  * the continuum closed forms for sin(kx) (Sec. 2.1 operator definitions), at the quadrature's
    order of accuracy;
  * polynomial exactness with Dirichlet data, against the continuum inverse written as a
    derivative series plus homogeneous solutions;
  * the truncation orders of the partial sums (Sec. 2.2, truncation statements);
  * the paper's nearest-neighbour block decomposition (Sec. 3.1-3.3) reproducing the global result
    within the tolerance eps = e^{-alpha L_m}.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle

OPS = ("L", "R", "0")


def _weights_R(nu, order):
    """J_R offsets m and weights (node x_{i+m} at eta = -m)."""
    ms = list(range(-3, 3)) if order == 6 else list(range(-2, 2))
    return ms, oracle.weights(nu, [-m for m in ms])


def _weights_L(nu, order):
    ms = list(range(-2, 4)) if order == 6 else list(range(-1, 3))
    return ms, oracle.weights(nu, ms)


def _symbols(nu, order, N):
    """Discrete symbols of L_L^{-1}, L_R^{-1}, L_0^{-1} on a periodic line of N points."""
    th = 2 * np.pi * np.arange(N) / N
    d = math.exp(-nu)
    mR, wR = _weights_R(nu, order)
    mL, wL = _weights_L(nu, order)
    WR = sum(w * np.exp(1j * th * m) for m, w in zip(mR, wR))
    WL = sum(w * np.exp(1j * th * m) for m, w in zip(mL, wL))
    sR = WR / (1 - d * np.exp(-1j * th))
    sL = WL / (1 - d * np.exp(1j * th))
    return {"L": sL, "R": sR, "0": 0.5 * (sL + sR)}


def _noise_line(N, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(N) / N
    eta = rng.standard_normal(N)
    box = sum(np.roll(eta, j) for j in range(-4, 5)) / 9.0
    return np.sin(2 * np.pi * x) + 0.05 * box


# ------------------------------------------------------------------------------------------ P2
@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("nu", [0.04, 1.0, 6.0])
def test_periodic_brute_force_sum(order, nu):
    N = 97
    dx = 1.0 / N
    alpha = nu / dx
    v = _noise_line(N, 3)
    JL, JR = oracle.line_quad("periodic", order, alpha, dx, v)
    d, mu = math.exp(-nu), math.exp(-nu * N)
    n = np.arange(N)
    ref = {}
    ref["R"] = np.array([np.sum(d ** n * JR[(i - n) % N]) for i in range(N)]) / (1 - mu)
    ref["L"] = np.array([np.sum(d ** n * JL[(i + n) % N]) for i in range(N)]) / (1 - mu)
    ref["0"] = 0.5 * (ref["R"] + ref["L"])
    for op in OPS:
        got = oracle.line_invL("periodic", op, order, alpha, dx, v)
        np.testing.assert_allclose(got, ref[op], rtol=0, atol=2e-15 * np.abs(ref[op]).max() * max(1, 1 / nu))


def _interp_cell(order, j, N, xs, v, bc):
    """Nodes (positions, values) of the interpolant used on cell [x_j, x_{j+1}]."""
    lo = j - 2 if order == 6 else j - 1
    if bc == "dirichlet":
        n = N + 1
        lo = max(0, min(lo, n - order))
        idx = list(range(lo, lo + order))
        return [xs[k] for k in idx], [v[k] for k in idx]
    dx = xs[1] - xs[0]
    idx = list(range(lo, lo + order))
    return [xs[0] + k * dx for k in idx], [v[k % N] for k in idx]


def _lag(px, pv, s):
    tot = mp.mpf(0)
    for a in range(len(px)):
        t = mp.mpf(pv[a])
        for b in range(len(px)):
            if b != a:
                t *= (s - px[b]) / (px[a] - px[b])
        tot += t
    return tot


@pytest.mark.parametrize("order", [4, 6])
def test_periodic_green_function_direct_integral(order):
    """L^{-1} at each node = integral of the periodic Green's function against the piecewise
    interpolant (the cell interpolant shared by J_R and J_L), by mpmath quadrature."""
    mp.mp.dps = 30
    N, L, nu = 11, 1.0, 0.7
    dx = L / N
    alpha = nu / dx
    xs = [mp.mpf(i) * mp.mpf(L) / N for i in range(N + 1)]
    v = list(_noise_line(N, 5))
    mu = mp.exp(-alpha * L)
    got = {op: oracle.line_invL("periodic", op, order, alpha, dx, np.array(v)) for op in OPS}
    for i in (0, 3, 10):
        xi = xs[i]
        acc = {op: mp.mpf(0) for op in OPS}
        for j in range(N):
            px, pv = _interp_cell(order, j, N, xs, v, "periodic")
            a, b = xs[j], xs[j + 1]
            left = b <= xi  # cell lies left of x_i
            gR = (lambda s: alpha * mp.exp(-alpha * (xi - s)) / (1 - mu)) if left else \
                 (lambda s: alpha * mp.exp(-alpha * (xi - s + L)) / (1 - mu))
            gL = (lambda s: alpha * mp.exp(-alpha * (s - xi)) / (1 - mu)) if not left else \
                 (lambda s: alpha * mp.exp(-alpha * (s - xi + L)) / (1 - mu))
            g0 = lambda s: 0.5 * alpha * (mp.exp(-alpha * abs(xi - s)) + mp.exp(-alpha * (L - abs(xi - s)))) / (1 - mu)
            for op, g in (("R", gR), ("L", gL), ("0", g0)):
                acc[op] += mp.quad(lambda s: g(s) * _lag(px, pv, s), [a, b])
        for op in OPS:
            assert abs(got[op][i] - float(acc[op])) < 5e-15, (op, i, got[op][i], float(acc[op]))


@pytest.mark.parametrize("order", [4, 6])
def test_dirichlet_direct_integral_and_end_values(order):
    mp.mp.dps = 30
    N, L, nu = 12, 1.0, 0.9
    n = N + 1
    dx = L / N
    alpha = nu / dx
    xs = [mp.mpf(i) * mp.mpf(L) / N for i in range(n)]
    v = list(np.cos(3.0 * np.arange(n) * dx) + 0.3 * np.arange(n) * dx)
    ga, gb = 0.25, -0.5
    mu = math.exp(-alpha * L)
    got = oracle.line_invL("dirichlet", "0", order, alpha, dx, np.array(v), ga, gb)
    I0 = []
    for xi in xs:
        acc = mp.mpf(0)
        for j in range(N):
            px, pv = _interp_cell(order, j, N, xs, v, "dirichlet")
            acc += mp.quad(lambda s: 0.5 * alpha * mp.exp(-alpha * abs(xi - s)) * _lag(px, pv, s), [xs[j], xs[j + 1]])
        I0.append(float(acc))
    M = np.array([[1.0, mu], [mu, 1.0]])
    A, B = np.linalg.solve(M, [ga - I0[0], gb - I0[-1]])
    x = np.arange(n) * dx
    ref = np.array(I0) + A * np.exp(-alpha * x) + B * np.exp(-alpha * (L - x))
    np.testing.assert_allclose(got, ref, rtol=0, atol=5e-15)
    assert abs(got[0] - ga) < 1e-15 and abs(got[-1] - gb) < 1e-15


# ------------------------------------------------------------------------------------------ P3
@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("nu", [0.039166, 1.0, 3.0])
def test_fft_symbol(order, nu):
    N = 1024
    dx = 1.0 / N
    v = _noise_line(N, 200703042)
    s = _symbols(nu, order, N)
    V = np.fft.fft(v)
    for op in OPS:
        ref = np.real(np.fft.ifft(V * s[op]))
        got = oracle.line_invL("periodic", op, order, nu / dx, dx, v)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14 * np.abs(v).max())
        # D partial sums: symbol (1 - s)^p
        for k in (1, 2, 3):
            sig = 1 - s[op]
            refk = np.real(np.fft.ifft(V * sum(sig ** p for p in range(1, k + 1))))
            gotk = oracle.apply_D_partial_sum(oracle.make_grid((N,)), 0, op, order, nu / dx, k, 1.0, v)
            np.testing.assert_allclose(gotk, refk, rtol=0, atol=1e-13 * np.abs(v).max())


# ------------------------------------------------------------------------------------------ P4
def _closed_form(op, alpha, k, x):
    s, c = np.sin(k * x), np.cos(k * x)
    den = alpha ** 2 + k ** 2
    if op == "0":
        return alpha ** 2 / den * s
    if op == "R":
        return alpha * (alpha * s - k * c) / den
    return alpha * (alpha * s + k * c) / den


@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("op", OPS)
def test_sin_closed_form_convergence(order, op):
    L, k, alpha = 2 * np.pi, 3.0, 12.0
    errs = []
    for N in (48, 96, 192):
        dx = L / N
        x = np.arange(N) * dx
        got = oracle.line_invL("periodic", op, order, alpha, dx, np.sin(k * x))
        errs.append(np.abs(got - _closed_form(op, alpha, k, x)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > order - 0.4, (errs, rates)


def test_config_one_sin_mode_matches_continuum():
    """N = 1024 on [0,1], alpha = 1024 (nu = 1): discrete L_0^{-1}[sin 2 pi x] = continuum value."""
    N = 1024
    dx = 1.0 / N
    x = np.arange(N) * dx
    k = 2 * np.pi
    for op in OPS:
        got = oracle.line_invL("periodic", op, 6, 1024.0, dx, np.sin(k * x))
        np.testing.assert_allclose(got, _closed_form(op, 1024.0, k, x), rtol=0, atol=2e-15)


# ------------------------------------------------------------------------------------------ P5
@pytest.mark.parametrize("n", [1, 2, 3])
def test_partial_sum_truncation_order_second_derivative(n):
    """-alpha^2 sum_{p<=n} D_0^p -> d_xx with error O(alpha^{-2n}) (Sec. 2.2)."""
    N, L, k = 1024, 2 * np.pi, 1.0
    dx = L / N
    x = np.arange(N) * dx
    g = oracle.make_grid((N,), (0.0,), (L,))
    alphas = [8.0, 16.0, 32.0]
    errs = []
    for a in alphas:
        S = oracle.apply_D_partial_sum(g, 0, "0", 6, a, n, -a * a, np.sin(k * x))
        errs.append(np.abs(S - (-k * k * np.sin(k * x))).max())
    slope = np.polyfit(np.log(alphas), np.log(errs), 1)[0]
    assert abs(slope + 2 * n) < 0.15, (errs, slope)


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("op", ["R", "L"])
def test_partial_sum_truncation_order_first_derivative(n, op):
    """alpha sum D_R^p -> d_x^- and -alpha sum D_L^p -> d_x^+, error O(alpha^{-n})."""
    N, L, k = 1024, 2 * np.pi, 1.0
    dx = L / N
    x = np.arange(N) * dx
    g = oracle.make_grid((N,), (0.0,), (L,))
    alphas = [16.0, 32.0, 64.0]
    errs = []
    for a in alphas:
        scale = a if op == "R" else -a
        S = oracle.apply_D_partial_sum(g, 0, op, 6, a, n, scale, np.sin(k * x))
        errs.append(np.abs(S - k * np.cos(k * x)).max())
    slope = np.polyfit(np.log(alphas), np.log(errs), 1)[0]
    assert abs(slope + n) < 0.15, (errs, slope)


def test_partial_sums_match_continuum_symbol():
    """S_n^0[sin kx] = q(1-q^n)/(1-q) sin kx with q = k^2/(alpha^2+k^2)."""
    N, L, k, a = 2048, 2 * np.pi, 2.0, 20.0
    dx = L / N
    x = np.arange(N) * dx
    g = oracle.make_grid((N,), (0.0,), (L,))
    q = k * k / (a * a + k * k)
    for n in (1, 2, 3):
        S = oracle.apply_D_partial_sum(g, 0, "0", 6, a, n, 1.0, np.sin(k * x))
        np.testing.assert_allclose(S, q * (1 - q ** n) / (1 - q) * np.sin(k * x), rtol=0, atol=1e-12)


# ------------------------------------------------------------------------------------------ P6
def _series(p, alpha, sign, even_only):
    """sum_m c^m p^{(m)} as a numpy polynomial (finite for polynomials)."""
    out = np.polynomial.Polynomial([0.0])
    dp = p
    m = 0
    while dp.degree() >= 0 and np.any(dp.coef != 0):
        if not even_only or m % 2 == 0:
            out = out + (sign / alpha) ** m * dp
        dp = dp.deriv()
        m += 1
        if m > 12:
            break
    return out


@pytest.mark.parametrize("order", [4, 6])
def test_dirichlet_polynomial_exactness(order):
    deg = order - 1
    rng = np.random.default_rng(11)
    p = np.polynomial.Polynomial(rng.uniform(-1, 1, deg + 1))
    N, L = 40, 1.0
    n = N + 1
    dx = L / N
    x = np.arange(n) * dx
    alpha = 9.0
    ga, gb = 0.3, -0.7
    mu = math.exp(-alpha * L)
    ea, eb = np.exp(-alpha * x), np.exp(-alpha * (L - x))
    v = p(x)
    # L_0 = I - alpha^-2 d_xx: particular solution sum_m alpha^{-2m} p^{(2m)}
    up = _series(p, alpha, 1.0, True)
    A, B = np.linalg.solve([[1, mu], [mu, 1]], [ga - up(0.0), gb - up(L)])
    ref0 = up(x) + A * ea + B * eb
    got0 = oracle.line_invL("dirichlet", "0", order, alpha, dx, v, ga, gb)
    np.testing.assert_allclose(got0, ref0, rtol=0, atol=1e-13 * np.abs(ref0).max())
    # L_R = I + alpha^-1 d_x: sum_m (-1/alpha)^m p^{(m)} + C e^{-alpha(x-a)}, value ga at a
    uR = _series(p, alpha, -1.0, False)
    refR = uR(x) + (ga - uR(0.0)) * ea
    gotR = oracle.line_invL("dirichlet", "R", order, alpha, dx, v, ga, gb)
    np.testing.assert_allclose(gotR, refR, rtol=0, atol=1e-13 * np.abs(refR).max())
    uL = _series(p, alpha, 1.0, False)
    refL = uL(x) + (gb - uL(L)) * eb
    gotL = oracle.line_invL("dirichlet", "L", order, alpha, dx, v, ga, gb)
    np.testing.assert_allclose(gotL, refL, rtol=0, atol=1e-13 * np.abs(refL).max())


def test_dirichlet_exponential_converges_at_order():
    """v = e^{lam x}: L_0^{-1} particular solution alpha^2/(alpha^2 - lam^2) e^{lam x}."""
    lam, alpha, L = 2.5, 7.0, 1.0
    errs = []
    for N in (32, 64, 128):
        dx = L / N
        x = np.arange(N + 1) * dx
        ga, gb = 0.0, 0.0
        mu = math.exp(-alpha * L)
        up = alpha ** 2 / (alpha ** 2 - lam ** 2) * np.exp(lam * x)
        A, B = np.linalg.solve([[1, mu], [mu, 1]], [ga - up[0], gb - up[-1]])
        ref = up + A * np.exp(-alpha * x) + B * np.exp(-alpha * (L - x))
        got = oracle.line_invL("dirichlet", "0", 6, alpha, dx, np.exp(lam * x), ga, gb)
        errs.append(np.abs(got - ref).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 5.5, (errs, rates)


# ------------------------------------------------------------------------------------------ P7
@pytest.mark.parametrize("op", OPS)
def test_nearest_neighbour_blocks_reproduce_global(op):
    """Sec. 3: each block sweeps locally from zero; the N-N constants (compact forms of Sec. 3.2 and
    3.3, periodic choice at the ends) reproduce the global operator within e^{-alpha L_m}."""
    N, nb, nu = 480, 6, 0.5
    M = N // nb  # block length in cells: alpha L_m = nu M = 40 -> e^{-40} < 1e-16
    dx = 1.0 / N
    alpha = nu / dx
    v = _noise_line(N, 9)
    JL, JR = oracle.line_quad("periodic", 6, alpha, dx, v)
    d = math.exp(-nu)
    IR, IL = [], []  # per block, arrays over the block's points iM..(i+1)M inclusive
    for i in range(nb):
        r = np.zeros(M + 1)
        for p in range(1, M + 1):
            r[p] = d * r[p - 1] + JR[(i * M + p) % N]
        l = np.zeros(M + 1)
        for p in range(M - 1, -1, -1):
            l[p] = d * l[p + 1] + JL[(i * M + p) % N]
        IR.append(r)
        IL.append(l)
    out = np.zeros(N)
    s = 0.5 if op == "0" else 1.0
    for i in range(nb):
        Ai = s * IR[(i - 1) % nb][M]   # previous block's right-moving integral at c_i
        Bi = s * IL[(i + 1) % nb][0]   # next block's left-moving integral at c_{i+1}
        p = np.arange(M)
        if op == "R":
            out[i * M:(i + 1) * M] = IR[i][:M] + Ai * d ** p
        elif op == "L":
            out[i * M:(i + 1) * M] = IL[i][:M] + Bi * d ** (M - p)
        else:
            out[i * M:(i + 1) * M] = 0.5 * (IL[i][:M] + IR[i][:M]) + Ai * d ** p + Bi * d ** (M - p)
    glob = oracle.line_invL("periodic", op, 6, alpha, dx, v)
    eps = math.exp(-nu * M)
    assert eps < 1e-16
    assert np.abs(out - glob).max() <= 4e-16 * np.abs(glob).max() + eps * np.abs(glob).max()


# ------------------------------------------------------------------------------------------ misc
def test_multi_dimensional_lines_follow_axis():
    """Applying along axis d equals applying the 1-D line operator to every line of that axis."""
    rng = np.random.default_rng(1)
    u = rng.standard_normal((5, 7, 9))
    g = oracle.make_grid((9, 7, 5), (0, 0, 0), (1.0, 2.0, 3.0), ("periodic", "dirichlet", "periodic"))
    gv = rng.standard_normal((5 * 9, 2))
    out1 = oracle.apply_invL(g, 1, "0", 4, 5.0, u, gv)
    dx = 2.0 / 6
    for z in range(5):
        for x in range(9):
            L = z * 9 + x
            ref = oracle.line_invL("dirichlet", "0", 4, 5.0, dx, u[z, :, x], gv[L, 0], gv[L, 1])
            np.testing.assert_array_equal(out1[z, :, x], ref)
    out2 = oracle.apply_invL(g, 2, "R", 4, 5.0, u)
    for y in range(7):
        for x in range(9):
            ref = oracle.line_invL("periodic", "R", 4, 5.0, 3.0 / 5, u[:, y, x])
            np.testing.assert_array_equal(out2[:, y, x], ref)


def test_large_nu_underflow_and_small_lines():
    v = np.linspace(-1, 1, 7)
    for bc in ("periodic", "dirichlet"):
        for op in OPS:
            out = oracle.line_invL(bc, op, 6, 400.0, 0.1, v)  # nu = 40, mu underflows
            assert np.all(np.isfinite(out))
    with pytest.raises(ValueError):
        oracle.line_invL("periodic", "0", 6, 1.0, 0.1, np.ones(6))  # fewer than order+1 points
