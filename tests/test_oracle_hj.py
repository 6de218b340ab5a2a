"""Pins of the nonlinear Hamilton-Jacobi oracle (oracle/hj.py) and of the MLP oracle (oracle/mlp.py)
against facts outside them: exact rational limits, closed forms, the continuum derivative symbol,
the characteristics of the exact solution, convergence orders and finite differences."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import hj, mlp


def lagrange_integrals(nodes):
    """int_0^1 l_j(eta) d eta for integer nodes, exactly (the nu -> 0 limit of weights / nu)."""
    out = []
    for j, a in enumerate(nodes):
        poly = [Fraction(1)]  # coefficients, ascending powers
        den = Fraction(1)
        for k, b in enumerate(nodes):
            if k == j:
                continue
            poly = [Fraction(0)] + poly  # * eta
            poly = [poly[i] - b * (poly[i + 1] if i + 1 < len(poly) else 0) for i in range(len(poly))]
            den *= (a - b)
        # note: the loop above multiplies by (eta - b) in ascending-power form
        out.append(sum(c / (i + 1) for i, c in enumerate(poly)) / den)
    return out


def test_lagrange_helper_on_known_rule():
    # nodes 0, 1: trapezoid on [0, 1]
    assert lagrange_integrals([0, 1]) == [Fraction(1, 2), Fraction(1, 2)]
    # Simpson-like check: nodes 0, 1, 2 integrate 1, eta, eta^2 exactly
    w = lagrange_integrals([0, 1, 2])
    assert sum(w) == 1 and sum(wi * n for wi, n in zip(w, [0, 1, 2])) == Fraction(1, 2)
    assert sum(wi * n * n for wi, n in zip(w, [0, 1, 2])) == Fraction(1, 3)


@pytest.mark.parametrize("nu", [1e-3, 0.05, 0.5, 1.0, 3.0])
def test_linear_weights_exist_and_form_a_partition_of_unity(nu):
    w5, c, d, res = hj.weno5_coefficients(nu)
    assert res < 1e-14 * np.abs(w5).max()
    assert abs(d.sum() - 1.0) < 1e-12
    assert (d > 0).all()
    # every rule integrates constants exactly: sum of weights = 1 - e^{-nu}
    for w in [w5, *c]:
        assert abs(w.sum() + math.expm1(-nu)) < 1e-14


def test_linear_weights_small_nu_limit_is_the_polynomial_rule():
    w5 = lagrange_integrals(list(hj.ETA5))
    subs = [lagrange_integrals(list(s)) for s in hj.SUB]
    d0 = w5[0] / subs[0][0]          # slot of eta = 3 only in S_0
    d2 = w5[4] / subs[2][2]          # slot of eta = -1 only in S_2
    d1 = 1 - d0 - d2
    _, _, d, _ = hj.weno5_coefficients(1e-7)
    for got, want in zip(d, (d0, d1, d2)):
        assert abs(got - float(want)) < 1e-5


def test_smoothness_is_the_squared_second_difference():
    r = np.random.default_rng(3)
    S = r.standard_normal((50, 5))
    b = hj.smoothness(S)
    for k in range(3):
        want = (S[:, k] - 2 * S[:, k + 1] + S[:, k + 2]) ** 2
        assert np.allclose(b[:, k], want, rtol=1e-12, atol=1e-14)


def test_wenoz_equals_linear_weights_on_quadratic_data():
    _, _, d, _ = hj.weno5_coefficients(0.7)
    eta = np.array(hj.ETA5, dtype=float)
    S = np.stack([0.3 * eta ** 2 - 1.2 * eta + 0.5, 2.0 * eta ** 2 + 7.0])
    om = hj.wenoz_weights(hj.smoothness(S), d)
    assert np.abs(om - d).max() < 1e-14


def test_wenoz_suppresses_the_substencil_across_a_kink():
    _, _, d, _ = hj.weno5_coefficients(1.0)
    dx = 0.01
    eta = np.array(hj.ETA5, dtype=float)
    x = -eta * dx  # node positions relative to x_i
    # kink between x_{i-3} and x_{i-2}: only S_0 contains both sides
    S = np.abs(x + 2.5 * dx)[None, :]
    om = hj.wenoz_weights(hj.smoothness(S), d)[0]
    # WENO-Z: the kinked substencil keeps ~ d_0 (1 + tau / beta_0) against d_r (1 + tau / eps) for the
    # smooth ones (tau ~ beta_0 ~ 1e-4 here): a 50-fold relative cut
    assert om[0] < 0.05 * d[0] and abs(om.sum() - 1) < 1e-15


@pytest.mark.parametrize("k", [1, 3])
def test_derivatives_match_the_continuum_symbol(k):
    """alpha D_R[sin kx] = alpha k (k sin + alpha cos) / (alpha^2 + k^2); -alpha D_L[sin kx] =
    alpha k (alpha cos - k sin) / (alpha^2 + k^2) (from the closed forms of L_R^{-1}, L_L^{-1}).
    The 5-point rule makes L^{-1} fifth-order accurate; the factor alpha = 1/dx leaves fourth order
    for the derivatives."""
    errs = []
    for n in (64, 128):
        L = 2 * math.pi
        dx = L / n
        x = np.arange(n) * dx
        alpha = 1.0 / dx
        v = np.sin(k * x)
        vm, vp = hj.derivatives(v, alpha, dx, "linear")
        s, c = np.sin(k * x), np.cos(k * x)
        wm = alpha * k * (k * s + alpha * c) / (alpha ** 2 + k ** 2)
        wp = alpha * k * (alpha * c - k * s) / (alpha ** 2 + k ** 2)
        errs.append(max(np.abs(vm - wm).max(), np.abs(vp - wp).max()) / k)
    assert errs[1] < 1e-5
    assert errs[0] / errs[1] > 2 ** 3.6


@pytest.mark.parametrize("t", [0.3, 0.9])
def test_hopf_lax_solution_follows_the_characteristics(t):
    """Before the kinks form (t < 1) the solution is w = sin y + t cos^2 y / 2 at x = y + t cos y."""
    y = np.linspace(-3.0, 3.0, 41)
    x = y + t * np.cos(y)
    w = hj.hopf_lax_1d(x, t)
    assert np.abs(w - (np.sin(y) + 0.5 * t * np.cos(y) ** 2)).max() < 1e-10


def test_hopf_lax_kink_after_crossing():
    """For t > 1 the solution has a kink (jump in w_x) where characteristics cross, at x = pi/2 + 2 pi k
    by symmetry of sin about pi/2 ... checked as a one-sided slope jump."""
    t = 1.5
    h = 1e-4
    xs = np.array([math.pi / 2 - 2 * h, math.pi / 2 - h, math.pi / 2, math.pi / 2 + h, math.pi / 2 + 2 * h])
    w = hj.hopf_lax_1d(xs, t)
    left, right = (w[2] - w[1]) / h, (w[3] - w[2]) / h
    assert abs(left - right) > 0.1


def test_hj_linear_scheme_converges_at_first_order():
    T = 0.5
    errs = []
    for n in (32, 64, 128):
        L = 2 * math.pi
        x = np.arange(n) * (L / n)
        u0 = np.sin(x)[None, :] + np.sin(x)[:, None]
        u, hist = hj.hj_run(u0, L, T, mode="linear")
        assert abs(hist[-1][0] - T) < 1e-12
        errs.append(np.abs(u - hj.exact_solution(n, n, L, T)).max())
    assert errs[0] / errs[1] > 1.6 and errs[1] / errs[2] > 1.6
    assert errs[2] < 1.5 * (2 * math.pi / 128)  # first order: about dx


def test_hj_nonlinear_weights_beat_linear_weights_after_kinks():
    n, T = 64, 1.5
    L = 2 * math.pi
    x = np.arange(n) * (L / n)
    u0 = np.sin(x)[None, :] + np.sin(x)[:, None]
    ex = hj.exact_solution(n, n, L, T)
    el = np.abs(hj.hj_run(u0, L, T, mode="linear")[0] - ex).max()
    ez = np.abs(hj.hj_run(u0, L, T, mode="wenoz")[0] - ex).max()
    assert ez < el


# ------------------------------------------------------------------------------ MLP oracle
def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-40, 65504.0])
    got = mlp.bf16(vals)
    assert got[0] == 1.0
    assert got[1] == 1.0                      # tie rounds to even (mantissa ...0)
    assert got[2] == 1.0 + 4 * 2 ** -8        # tie rounds to even (up)
    assert got[3] == -2.5
    assert got[5] == 65536.0


def test_features_are_shift_and_scale_invariant_except_the_scale_feature():
    r = np.random.default_rng(5)
    S = r.standard_normal((20, 5))
    f = mlp.features(S)
    g = mlp.features(3.0 * S + 7.0)
    inv = [0, 1, 2, 4, 5, 6, 7]
    assert np.allclose(f[:, inv], g[:, inv], atol=1e-14)
    unclipped = (np.abs(f[:, 3]) < 0.99) & (np.abs(g[:, 3]) < 0.99)
    assert unclipped.any()
    assert np.allclose((g[:, 3] - f[:, 3])[unclipped], math.log10(9.0) / 8, atol=1e-12)
    assert (np.abs(f) <= 1 + 1e-15).all()
    # second differences: a quadratic stencil has q_0 = q_1 = q_2
    eta = np.array(hj.ETA5, dtype=float)
    fq = mlp.features((0.4 * eta ** 2 - eta)[None, :])
    assert np.allclose(fq[0, :3], np.sign(0.8) * np.ones(3))
    c = mlp.features(np.ones((1, 5)))
    assert np.all(c[:, [0, 1, 2, 4, 5, 6, 7]] == 0) and c[0, 3] == -1.0


def test_mlp_gradients_match_central_differences():
    """Backward against central differences of the loss (FP64)."""
    r = np.random.default_rng(9)
    p = mlp.init_params(1)
    for k in p:
        p[k] = p[k] + 0.05 * r.standard_normal(p[k].shape)
    X = mlp.features(r.standard_normal((16, 5)))
    T = r.dirichlet(np.ones(3), 16)
    om, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, T)
    h = 1e-6
    for k in p:
        idx = [tuple(r.integers(0, s) for s in p[k].shape) for _ in range(3)]
        for ix in idx:
            if k == "W1" and ix[1] >= 6:
                continue
            pp = {q: v.copy() for q, v in p.items()}
            pm = {q: v.copy() for q, v in p.items()}
            pp[k][ix] += h
            pm[k][ix] -= h
            fd = (mlp.loss(mlp.forward(pp, X)[0], T) - mlp.loss(mlp.forward(pm, X)[0], T)) / (2 * h)
            assert abs(fd - g[k][ix]) < 1e-7 + 1e-5 * abs(fd), (k, ix, fd, g[k][ix])


def _adam_scalar(p0, grads, lr, **kw):
    p = {"w": np.array([p0], dtype=float)}
    st = {}
    for g in grads:
        mlp.adam_step(p, {"w": np.array([g], dtype=float)}, st, lr, **kw)
    return float(p["w"][0]), st


def test_adam_step_pinned_by_hand_derived_values():
    """Adam (Kingma & Ba) at b1 = 0.9, b2 = 0.999, eps = 1e-8, values worked out by hand:
    * step 1 from zero moments: m = 0.1 g, v = 0.001 g^2, the bias corrections give m^ = g,
      v^ = g^2, so the parameter moves by -lr g / (|g| + eps);
    * a constant gradient keeps m^ = g and v^ = g^2 at every step (the corrections divide by
      1 - b^t exactly what the moments lack), so each step moves by the same amount;
    * g = 1 then g = -1: m^ = (0.9 - 1) / 1.9 = -1/19, v^ = (0.999 + 1) / 1.999 = 1, so the second
      step moves by +lr / (19 (1 + eps));
    * a gradient of the size of eps: step 1 moves by -lr g / (g + eps) = -lr / 2 at g = eps
      (eps outside the square root).
    A dropped or misplaced bias correction, a swapped b1/b2 or eps inside the root fails one."""
    lr, eps = 0.1, 1e-8
    for g in (3.0, -0.25, 1e4):
        w, st = _adam_scalar(0.5, [g], lr)
        assert abs(w - (0.5 - lr * g / (abs(g) + eps))) < 1e-15
        assert st["t"] == 1
        assert abs(st["m_w"][0] - 0.1 * g) < 1e-15 * abs(g) and abs(st["v_w"][0] - 1e-3 * g * g) < 1e-15 * g * g
    w, st = _adam_scalar(0.0, [2.0] * 5, lr)
    assert abs(w - (-5 * lr * 2.0 / (2.0 + eps))) < 1e-14 and st["t"] == 5
    w, _ = _adam_scalar(0.0, [1.0, -1.0], lr)
    assert abs(w - (-lr / (1 + eps) + lr / (19 * (1 + eps)))) < 1e-15
    w, _ = _adam_scalar(0.0, [eps], lr)
    assert abs(w - (-lr / 2)) < 1e-15
    # without the bias corrections step 1 would move by lr 0.1 / sqrt(0.001) = 3.16 lr: the pin above
    # is a factor 3 away from that mistake
    assert abs(0.1 / math.sqrt(1e-3) - 1.0) > 2


def test_adam_decreases_the_loss_on_a_fixed_batch():
    r = np.random.default_rng(2)
    p = mlp.init_params(3)
    X = mlp.features(r.standard_normal((256, 5)))
    T = r.dirichlet(np.ones(3), 256)
    st = {}
    l0 = mlp.loss(mlp.forward(p, X)[0], T)
    for _ in range(200):
        om, c = mlp.forward(p, X)
        mlp.adam_step(p, mlp.backward(p, c, T), st, 3e-3)
    assert mlp.loss(mlp.forward(p, X)[0], T) < 0.5 * l0


# ------------------------------------------------------------------------------ Example 3, per-axis speeds
def test_example3_manufactured_solution_converges_first_order():
    """Sec. 5.1, Example 3: u_t + (1 + u_x + u_y)^2 / 2 = S on [0, 2 pi]^2, u0 = 0, T = 0.5, linear
    weights, the adaptive rule with the lagged wave speeds; with the source of the manufactured
    solution u = t (sin x + sin y) the error falls at first order (the Euler step), and the tracked
    wave speed approaches max |1 + u_x + u_y| = 1 + 2T."""
    L, T = 2 * math.pi, 0.5
    errs = []
    for n in (64, 128, 256):
        u, hist = hj.hj_run_general(np.zeros((n, n)), L, T, cfl=1.0, kind="ex3", source=hj.example3_source)
        x = np.arange(n) * (L / n)
        exact = T * (np.sin(x)[None, :] + np.sin(x)[:, None])
        errs.append(np.abs(u - exact).max())
        assert abs(hist[-1][0] - T) < 1e-14
        assert abs(hist[-1][2] - (1 + 2 * T)) < 0.05 * (1 + 2 * T)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert errs[0] > errs[1] > errs[2]
    assert 0.8 < rates[-1] < 1.3, rates
    assert errs[-1] < 0.015


def test_per_axis_speeds_reduce_to_the_symmetric_rule():
    """With equal speeds on equal spacings (u0 = sin x + sin y) the per-axis rule takes the same
    steps, alpha and dissipation as the one-speed rule, so the two runs agree to rounding."""
    L, T, n = 2 * math.pi, 0.75, 48
    x = np.arange(n) * (L / n)
    u0 = np.sin(x)[None, :] + np.sin(x)[:, None]
    a, ha = hj.hj_run(u0, L, T, mode="linear")
    b, hb = hj.hj_run_general(u0, L, T, kind="quadratic", mode="linear")
    assert len(ha) == len(hb)
    assert np.abs(a - b).max() < 1e-12


def test_per_axis_speeds_on_unequal_speeds_follow_hopf_lax():
    """u0 = sin x + 0.3 sin y: the x speed is about three times the y speed; the per-axis rule
    (dt from the faster axis, alpha_y = beta / (c_y dt)) converges to the separable Hopf-Lax
    solution w_1(x, t) + w_{0.3}(y, t) before kinks form, and its y speed tracks max |u_y|."""
    L, T = 2 * math.pi, 0.5
    errs = []
    for n in (32, 64, 128):
        x = np.arange(n) * (L / n)
        u0 = np.sin(x)[None, :] + 0.3 * np.sin(x)[:, None]
        u, hist = hj.hj_run_general(u0, L, T, kind="quadratic", mode="linear")
        exact = hj.hopf_lax_1d(x, T)[None, :] + hj.hopf_lax_1d(x, T, amp=0.3)[:, None]
        errs.append(np.abs(u - exact).max())
        cx, cy = hist[-1][2], hist[-1][3]
        assert 2.5 < cx / cy < 4.0
    assert errs[0] > errs[1] > errs[2]
    assert math.log2(errs[1] / errs[2]) > 0.7
