"""Oracle of the nonlinear Hamilton-Jacobi example: WENO local quadrature, Lax-Friedrichs numerical
Hamiltonian, adaptive explicit steps.  Plain numpy, FP64.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT (same rules as the package: only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may use it).  The sweeps are the
C oracle's (``line_sweep``); everything else is written out here in the paper's order.

Readings (the paper gives the nonlinear quadrature only in outline, Sec. 2.4, and cites prior work
for the details):
  * 5-point quadrature from three 3-point substencils.  J_R[i] integrates the cell [x_{i-1}, x_i]
    against nu e^{-nu eta} (eta = distance from x_i in units of dx) over the nodes x_{i-3}..x_{i+1};
    substencil S_r = {x_{i-3+r}, x_{i-2+r}, x_{i-1+r}}, r = 0, 1, 2.  J_L is the mirror image
    (cell [x_i, x_{i+1}], nodes x_{i+3}..x_{i-1}).
  * Linear weights d_r: the partition of unity with sum_r d_r J^(r) = J^(5-point) (Sec. 2.4, the
    linear-weight combination), solved here by least squares over the 5 node coefficients.
  * Smoothness of substencil r: beta_r = sum_{l >= 2} dx^{2l-3} int_cell (p_r^(l))^2 dx over the
    derivative orders the interpolant has (the paper's commented indicator starts at l = 2; for the
    quadratic p_r only l = 2 remains).
  * Nonlinear weights: WENO-Z, w~_r = d_r (1 + tau / (eps + beta_r)), tau = |beta_0 - beta_2|,
    eps = 1e-6, normalised to sum 1.
  * Lax-Friedrichs Hamiltonian (Sec. 2.5): H^(v-, v+) = H((v- + v+)/2) + r (v- - v+)/2 per axis,
    r = the global max |H_p| (lagged), with v- = alpha D_R[u], v+ = -alpha D_L[u] (s = 1).
  * Adaptive step (the paper's adaptive rule with one lagged wave speed, as its adaptive examples
    keep the wave speeds symmetric): c = max over both axes of the one-sided derivatives of the
    previous step (initially of periodic central differences of u0), dt = CFL min(dx, dy) / c,
    alpha = beta / (c dt) = beta / (CFL min(dx, dy)) on both axes -- constant, so the quadrature
    weights are fixed -- and the Lax-Friedrichs coefficient r = c on both axes.
"""
from __future__ import annotations

import math

import numpy as np

from . import line_sweep, weights

ETA5 = (3, 2, 1, 0, -1)                      # node x_{i+m} <-> eta = -m
SUB = ((3, 2, 1), (2, 1, 0), (1, 0, -1))     # substencils, as eta positions
EPS_Z = 1e-6


def weno5_coefficients(nu: float):
    """(w5, c[3][3], d[3], residual): 5-point weights, substencil weights and linear weights."""
    w5 = weights(nu, ETA5)
    c = np.array([weights(nu, s) for s in SUB])
    A = np.zeros((5, 3))
    for r in range(3):
        A[r:r + 3, r] = c[r]
    d = np.linalg.lstsq(A, w5, rcond=None)[0]
    return w5, c, d, float(np.abs(A @ d - w5).max())


def smoothness(vals: np.ndarray) -> np.ndarray:
    """beta_r of the quadratic through the 3 values of each substencil (last axis: the 5 stencil
    values in ETA5 order), as the integral over the cell of the squared second derivative in
    scaled units (dx^{2l-3} int (p^(l))^2 dx with l = 2)."""
    out = []
    for r, s in enumerate(SUB):
        eta = np.array(s, dtype=float)
        y = vals[..., r:r + 3]
        # quadratic through (eta_j, y_j); its second eta-derivative is constant
        V = np.vander(eta, 3)            # columns eta^2, eta, 1
        coef = np.linalg.solve(V, np.moveaxis(y, -1, 0).reshape(3, -1))  # (3, m)
        p2 = 2.0 * coef[0]               # d^2 p / d eta^2
        # dx^{1} int_{cell} (d^2p/dx^2)^2 dx = int_0^1 (d^2 p / d eta^2)^2 d eta
        out.append((p2 ** 2).reshape(y.shape[:-1]))
    return np.stack(out, axis=-1)


def wenoz_weights(beta: np.ndarray, d: np.ndarray, eps: float = EPS_Z) -> np.ndarray:
    tau = np.abs(beta[..., 0] - beta[..., 2])[..., None]
    wt = d * (1.0 + tau / (eps + beta))
    return wt / wt.sum(axis=-1, keepdims=True)


def stencils(v: np.ndarray, mirror: bool) -> np.ndarray:
    """(n, 5) stencil values of a periodic line in ETA5 order: J_R uses x_{i+m}, m = -eta;
    J_L the mirror x_{i-m}."""
    n = v.size
    idx = np.arange(n)[:, None]
    m = -np.array(ETA5)[None, :]
    return v[(idx - m) % n] if mirror else v[(idx + m) % n]


def line_quad_weno(v: np.ndarray, nu: float, mode: str, omega=None):
    """(JL, JR, omega_L, omega_R) of a periodic line; mode 'linear' | 'wenoz' | 'given' (omega =
    (omega_L, omega_R) supplied by the caller)."""
    _, c, d, _ = weno5_coefficients(nu)
    res = []
    for k, mirror in enumerate((True, False)):
        S = stencils(v, mirror)
        if mode == "linear":
            om = np.broadcast_to(d, (v.size, 3))
        elif mode == "wenoz":
            om = wenoz_weights(smoothness(S), d)
        else:
            om = omega[k]
        Jr = np.stack([S[:, r:r + 3] @ c[r] for r in range(3)], axis=-1)
        res.append(((om * Jr).sum(axis=-1), om))
    (JL, oL), (JR, oR) = res
    return JL, JR, oL, oR


def derivatives(v: np.ndarray, alpha: float, dx: float, mode: str, omega=None):
    """(v-, v+) = (alpha D_R[v], -alpha D_L[v]) on a periodic line (Sec. 2.2, 2.3, 2.5)."""
    n = v.size
    JL, JR, _, _ = line_quad_weno(v, alpha * dx, mode, omega)
    IL, IR, ends = line_sweep("periodic", alpha, dx, JL, JR)
    d = math.exp(-alpha * dx)
    mu = math.exp(-alpha * dx * n)
    i = np.arange(n)
    LR = IR + ends[1] / (1.0 - mu) * d ** i
    LL = IL + ends[0] / (1.0 - mu) * d ** (n - i)
    return alpha * (v - LR), -alpha * (v - LL)


def hamiltonian(p, q, kind: str = "quadratic"):
    """H(p, q): 'quadratic' (p^2 + q^2) / 2 (the workload's equation) or 'ex3' (1 + p + q)^2 / 2
    (Example 3 of Sec. 5.1)."""
    if kind == "quadratic":
        return 0.5 * (p * p + q * q)
    s = 1.0 + p + q
    return 0.5 * s * s


def hamiltonian_lf(pm, pp, qm, qp, rx, ry, kind: str = "quadratic"):
    """Lax-Friedrichs numerical Hamiltonian (Sec. 2.5): H at the averages of the one-sided
    derivatives plus rx (p- - p+) / 2 + ry (q- - q+) / 2."""
    p, q = 0.5 * (pm + pp), 0.5 * (qm + qp)
    return hamiltonian(p, q, kind) + rx * 0.5 * (pm - pp) + ry * 0.5 * (qm - qp)


def wave_speeds(pm, pp, qm, qp, kind: str = "quadratic"):
    """(c_x, c_y) = (max |H_p|, max |H_q|) over the one-sided derivatives of a step."""
    if kind == "quadratic":
        return (float(max(np.abs(pm).max(), np.abs(pp).max())), float(max(np.abs(qm).max(), np.abs(qp).max())))
    # H_p = H_q = 1 + p + q: its largest magnitude over the four one-sided combinations
    m = max(float(np.abs(1.0 + a + b).max()) for a in (pm, pp) for b in (qm, qp))
    return m, m


def example3_source(x, y, t):
    """Source of Example 3 (Sec. 5.1) for the manufactured solution u = t (sin x + sin y):
    u_t + (1 + u_x + u_y)^2 / 2 = S with S = sin x + sin y + (1 + t cos x + t cos y)^2 / 2."""
    return np.sin(x) + np.sin(y) + 0.5 * (1.0 + t * np.cos(x) + t * np.cos(y)) ** 2


def hj_run_general(u0: np.ndarray, L: float, T: float, cfl: float = 1.0, beta: float = 1.0,
                   kind: str = "quadratic", source=None, mode: str = "linear", max_steps: int = 100000):
    """Forward-Euler steps of u_t + H(u_x, u_y) = S(x, y, t) on a periodic [0, L]^2 grid with the
    adaptive rule of Sec. 4.5 with one wave speed per axis:
      dt = CFL min(dx / c_x, dy / c_y),  alpha_x = beta / (c_x dt),  alpha_y = beta / (c_y dt)
    (the alpha choice of Example 1 with the step's own dt and speeds, so the quadrature weights
    change from step to step), Lax-Friedrichs coefficients c_x, c_y; the speeds of a step are the
    largest |H_p|, |H_q| of the previous step's one-sided derivatives (lagged; initially of periodic
    central differences of u0).  S is evaluated at the old time.  Returns (u, [(t, dt, c_x, c_y)])."""
    u = np.array(u0, dtype=float)
    ny, nx = u.shape
    dx, dy = L / nx, L / ny
    x = np.arange(nx) * dx
    y = np.arange(ny) * dy
    px = (np.roll(u, -1, axis=1) - np.roll(u, 1, axis=1)) / (2 * dx)
    py = (np.roll(u, -1, axis=0) - np.roll(u, 1, axis=0)) / (2 * dy)
    cx, cy = wave_speeds(px, px, py, py, kind)
    t, hist = 0.0, []
    for _ in range(max_steps):
        if t >= T - 1e-14:
            break
        dt = min(cfl * min(dx / cx, dy / cy), T - t)
        # alpha from the rule's full step (the last, shortened step keeps it)
        dt_rule = cfl * min(dx / cx, dy / cy)
        ax, ay = beta / (cx * dt_rule), beta / (cy * dt_rule)
        pm = np.empty_like(u)
        pp = np.empty_like(u)
        qm = np.empty_like(u)
        qp = np.empty_like(u)
        for j in range(ny):
            pm[j], pp[j] = derivatives(u[j], ax, dx, mode)
        for i in range(nx):
            qm[:, i], qp[:, i] = derivatives(u[:, i].copy(), ay, dy, mode)
        rhs = hamiltonian_lf(pm, pp, qm, qp, cx, cy, kind)
        if source is not None:
            rhs = rhs - source(x[None, :], y[:, None], t)
        u = u - dt * rhs
        t += dt
        cx, cy = wave_speeds(pm, pp, qm, qp, kind)
        hist.append((t, dt, cx, cy))
    return u, hist


def hj_run(u0: np.ndarray, L: float, T: float, cfl: float = 1.0, beta: float = 1.0, mode: str = "linear",
           omega_fn=None, max_steps: int = 100000):
    """Forward-Euler steps of u_t + (u_x^2 + u_y^2)/2 = 0 on a periodic [0, L]^2 grid (shape (ny, nx))
    up to time T (the last step shortened to land on T) with the adaptive lagged rule.
    omega_fn(stencils) -> weights for mode 'given'.  Returns (u, [(t, dt, c) per step])."""
    u = np.array(u0, dtype=float)
    ny, nx = u.shape
    dx, dy = L / nx, L / ny
    h = min(dx, dy)
    # initial wave speed from the initial condition (no lag yet): periodic central differences
    px = (np.roll(u, -1, axis=1) - np.roll(u, 1, axis=1)) / (2 * dx)
    py = (np.roll(u, -1, axis=0) - np.roll(u, 1, axis=0)) / (2 * dy)
    c = float(max(np.abs(px).max(), np.abs(py).max()))
    t, hist = 0.0, []
    ax = ay = beta / (cfl * h)
    for _ in range(max_steps):
        if t >= T - 1e-14:
            break
        dt = min(cfl * h / c, T - t)
        pm = np.empty_like(u)
        pp = np.empty_like(u)
        qm = np.empty_like(u)
        qp = np.empty_like(u)
        for j in range(ny):
            om = None if omega_fn is None else (omega_fn(stencils(u[j], True)), omega_fn(stencils(u[j], False)))
            pm[j], pp[j] = derivatives(u[j], ax, dx, mode, om)
        for i in range(nx):
            col = u[:, i].copy()
            om = None if omega_fn is None else (omega_fn(stencils(col, True)), omega_fn(stencils(col, False)))
            qm[:, i], qp[:, i] = derivatives(col, ay, dy, mode, om)
        Hh = hamiltonian_lf(pm, pp, qm, qp, c, c)
        u = u - dt * Hh
        t += dt
        # wave speed for the next step (lagged): max |H_p|, |H_q| over the one-sided derivatives
        c = float(max(np.abs(pm).max(), np.abs(pp).max(), np.abs(qm).max(), np.abs(qp).max()))
        hist.append((t, dt, c))
    return u, hist


def hopf_lax_1d(x: np.ndarray, t: float, nquad: int = 20001, amp: float = 1.0) -> np.ndarray:
    """Viscosity solution of w_t + w_x^2 / 2 = 0, w(x, 0) = amp sin x: w(x, t) = min_y amp sin y +
    (x - y)^2 / (2t), minimised over a fine grid around every x and refined by golden-section search."""
    if t == 0.0:
        return amp * np.sin(x)
    out = np.empty_like(x)
    span = math.pi * 1.05 + t
    ys = np.linspace(-span, span, nquad)
    for k, xv in enumerate(x):
        f = amp * np.sin(xv + ys) + ys ** 2 / (2 * t)
        j = int(np.argmin(f))
        a, b = xv + ys[max(j - 1, 0)], xv + ys[min(j + 1, nquad - 1)]
        g = (math.sqrt(5) - 1) / 2
        fn = lambda y: amp * math.sin(y) + (xv - y) ** 2 / (2 * t)
        c, d_ = b - g * (b - a), a + g * (b - a)
        for _ in range(80):
            if fn(c) < fn(d_):
                b = d_
            else:
                a = c
            c, d_ = b - g * (b - a), a + g * (b - a)
        out[k] = fn(0.5 * (a + b))
    return out


def exact_solution(nx: int, ny: int, L: float, t: float) -> np.ndarray:
    """u = w(x, t) + w(y, t) for u0 = sin x + sin y (the Hamiltonian separates)."""
    x = np.arange(nx) * (L / nx)
    y = np.arange(ny) * (L / ny)
    return hopf_lax_1d(y, t)[:, None] + hopf_lax_1d(x, t)[None, :]
