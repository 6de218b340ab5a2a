"""Pins of the oracle's quadrature weights (CPU only).

The oracle integrates kernel x Lagrange basis numerically (composite Gauss-Legendre, long double).
These tests tie it to things outside itself:
  * the closed-form coefficients printed in the paper's Appendix C (golden fixture, with the two
    misprints read as documented there), evaluated at 40 digits with mpmath;
  * the exact moments E_q(nu) = nu int_0^1 e^{-nu eta} eta^q d eta (analytic, mpmath), i.e.
    polynomial exactness of degree <= stencil width - 1 (Sec. 2.4: interpolation on the stencil);
  * the sum rule sum_j w_j = 1 - e^{-nu};
  * the nu -> 0 textbook limits (Adams-Moulton, centred four-point and six-point Newton-Cotes-type
    rules over one cell);
  * the mirror symmetry of J_L and J_R (Appendix C, last paragraph).
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "appendix_c_coefficients.txt")

ETA_SUB = {0: [3, 2, 1, 0], 1: [2, 1, 0, -1], 2: [1, 0, -1, -2]}  # S_r nodes x_{i-3+r..i+r}
ETA6 = [3, 2, 1, 0, -1, -2]  # J_R six-point stencil x_{i-3..i+2}; node x_{i+m} at eta = -m


def _appc():
    rows = {}
    with open(GOLD) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, num, den, tag = [t.strip() for t in line.split("|")]
            rows[name] = (num, den, tag)
    return rows


def _eval(expr_num, expr_den, nu):
    mp.mp.dps = 40
    env = {"n": mp.mpf(nu), "E": mp.exp(-mp.mpf(nu))}
    return eval(expr_num, {}, env) / eval(expr_den, {}, env)


def _appc_sub(nu, r, rows, printed=False):
    names = {0: ["c0_m3", "c0_m2", "c0_m1", "c0_0"], 1: ["c1_m2", "c1_m1", "c1_0", "c1_1"],
             2: ["c2_m1", "c2_0", "c2_1", "c2_2"]}[r]
    out = []
    for nm in names:
        if printed and nm + "_printed" in rows:
            nm = nm + "_printed"
        num, den, _ = rows[nm]
        out.append(_eval(num, den, nu))
    return out


@pytest.mark.parametrize("nu", [0.05, 0.3, 1.0, 2.5, 7.0])
@pytest.mark.parametrize("r", [0, 1, 2])
def test_substencil_weights_match_appendix_c(nu, r):
    rows = _appc()
    ref = np.array([float(x) for x in _appc_sub(nu, r, rows)])
    got = oracle.weights(nu, ETA_SUB[r])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-15 * np.abs(ref).max())


@pytest.mark.parametrize("nu", [0.05, 0.3, 1.0, 2.5, 7.0])
def test_six_point_weights_are_linear_weight_combination(nu):
    """Eq. (WENO linear weights): J_R = sum_r d_r J_R^{(r)} with the printed d_2 and the corrected d_0."""
    rows = _appc()
    c = [_appc_sub(nu, r, rows) for r in range(3)]
    d0 = _eval(*rows["d0"][:2], nu)
    d2 = _eval(*rows["d2"][:2], nu)
    d1 = 1 - d0 - d2
    d = [d0, d1, d2]
    w = [mp.mpf(0)] * 6
    for r in range(3):
        for j in range(4):
            w[r + j] += d[r] * c[r][j]
    ref = np.array([float(x) for x in w])
    got = oracle.weights(nu, ETA6)
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-15 * np.abs(ref).max())
    assert all(float(x) > 0 for x in d), "linear weights are positive (Sec. 2.4)"


def test_appendix_c_misprints_are_misprints():
    """The printed c^{(0)}_{-1} agrees with the integral only at nu = 1 (where nu^2 = nu^3); the printed
    d_0 does not reproduce the six-point rule at any nu (it tends to 1/2, not 11/60, as nu -> 0)."""
    rows = _appc()
    for nu in (0.3, 2.0):
        printed = float(_appc_sub(nu, 0, rows, printed=True)[2])
        assert abs(printed - oracle.weights(nu, ETA_SUB[0])[2]) > 1e-3
    printed1 = float(_appc_sub(1.0, 0, rows, printed=True)[2])
    assert abs(printed1 - oracle.weights(1.0, ETA_SUB[0])[2]) < 1e-15
    assert abs(float(_eval(*rows["d0_printed"][:2], 1e-3)) - 0.5) < 1e-3
    assert abs(float(_eval(*rows["d0"][:2], 1e-3)) - 11 / 60) < 1e-3


def _moment(q, nu):
    """E_q(nu) = nu int_0^1 e^{-nu t} t^q dt, exact (mpmath, 40 digits)."""
    mp.mp.dps = 40
    nu = mp.mpf(nu)
    return mp.factorial(q) / nu ** q * (1 - mp.exp(-nu) * sum(nu ** j / mp.factorial(j) for j in range(q + 1)))


@pytest.mark.parametrize("nu", [0.01, 0.039166, 0.5, 1.0, 4.0, 20.0])
@pytest.mark.parametrize("eta", [ETA6, [2, 1, 0, -1], [0, -1, -2, -3, -4, -5], [5, 4, 3, 2, 1, 0]])
def test_polynomial_exactness(nu, eta):
    w = oracle.weights(nu, eta)
    for q in range(len(eta)):
        ref = float(_moment(q, nu))
        got = float(sum(mp.mpf(wj) * mp.mpf(e) ** q for wj, e in zip(w, eta)))
        scale = float(sum(abs(wj) * abs(e) ** q for wj, e in zip(w, eta)))
        assert abs(got - ref) <= 4e-16 * max(scale, abs(ref)), (q, got, ref)


@pytest.mark.parametrize("nu", [1e-4, 0.039166, 1.0, 30.0])
def test_sum_rule(nu):
    for eta in (ETA6, [2, 1, 0, -1]):
        w = oracle.weights(nu, eta)
        ref = -math.expm1(-nu)
        assert abs(w.sum() - ref) <= 4e-16 * np.abs(w).sum(), (w.sum(), ref)


def test_small_nu_textbook_limits():
    nu = 1e-8
    lim = {
        (3, 2, 1, 0): np.array([1, -5, 19, 9]) / 24,  # Adams-Moulton over the last cell
        (2, 1, 0, -1): np.array([-1, 13, 13, -1]) / 24,
        (1, 0, -1, -2): np.array([9, 19, -5, 1]) / 24,
        tuple(ETA6): np.array([11, -93, 802, 802, -93, 11]) / 1440,
    }
    for eta, ref in lim.items():
        np.testing.assert_allclose(oracle.weights(nu, list(eta)) / nu, ref, rtol=0, atol=1e-7)


def test_mirror_symmetry_of_left_and_right_integrals():
    """J_L of a line equals J_R of the reversed line, reversed (Appendix C, mirror symmetry)."""
    rng = np.random.default_rng(7)
    for order in (4, 6):
        v = rng.standard_normal(37)
        JL, _ = oracle.line_quad("periodic", order, 3.0, 0.1, v)
        _, JRrev = oracle.line_quad("periodic", order, 3.0, 0.1, v[::-1].copy())
        np.testing.assert_allclose(JL, JRrev[::-1], rtol=0, atol=1e-15)
        JLd, _ = oracle.line_quad("dirichlet", order, 3.0, 0.1, v)
        _, JRdrev = oracle.line_quad("dirichlet", order, 3.0, 0.1, v[::-1].copy())
        # Dirichlet: J_L[i] covers [x_i, x_{i+1}], J_R[i+1] of the reversed line the mirrored cell
        np.testing.assert_allclose(JLd[:-1], JRdrev[::-1][:-1], rtol=0, atol=1e-15)
