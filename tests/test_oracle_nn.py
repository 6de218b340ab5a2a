"""Pins of the oracle's nearest-neighbour block form of L^{-1} (Sec. 3) against things outside it (CPU).

  * the N-N window invariant: with every block at least K = ceil(ln(1/eps) / nu) points long, the
    block form equals the global operator within eps * max|I| (Sec. 3.1, eq. (NN constraint
    general));
  * brute force: with short blocks (the truncation is large), every point equals the explicit sum of
    the local integrals J in its own block and its upstream neighbour block (cyclically for periodic
    lines, the wrapped cell counted with the last block), at their exact decay distances, plus the
    end-value terms; never touches the recurrences;
  * one periodic block: the block form and the global operator differ by exactly the geometric series
    of wraps beyond the first, A mu / (1 - mu) e^{-alpha (x - a)} (Sec. 2.3 periodic constants).
"""
import math

import numpy as np
import pytest

import oracle

OPS = ("L", "R", "0")


def _line(n, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(n) / n
    return np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x + 0.4) + 0.05 * rng.standard_normal(n)


def _dx(bc, n):
    return 1.0 / n if bc == "periodic" else 1.0 / (n - 1)


# ------------------------------------------------------------------------------------------ P7
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("nu,n,block", [(1.0, 296, 37), (0.5, 640, 80), (2.0, 412, 30)])
def test_window_invariant_within_eps(bc, op, nu, n, block):
    """Blocks of K >= ln(1/eps)/nu points (the last one ragged but at least K long): the N-N block
    form equals the global operator within (eps + rounding) * max|I|, eps = e^{-nu K}."""
    eps = 1e-16
    K = math.ceil(math.log(1 / eps) / nu)
    Lm = min(block, n % block or block)  # the shortest block
    assert Lm >= K
    dx = _dx(bc, n)
    alpha = nu / dx
    v = _line(n, 3)
    ga, gb = (0.7, -0.4) if bc == "dirichlet" else (0.0, 0.0)
    glob = oracle.line_invL(bc, op, 6, alpha, dx, v, ga, gb)
    nn = oracle.line_invL_nn(bc, op, 6, alpha, dx, v, block, ga, gb)
    scale = np.abs(glob).max()
    assert np.abs(nn - glob).max() <= (math.exp(-nu * Lm) + 4e-15) * scale


def _windows(bc, n, block, nu, JL, JR):
    """The right- and left-moving integrals of the block form written as explicit sums: point i of
    block b sees the J of its own block on its upwind side and all of its upstream neighbour block.
    Periodic: neighbours are cyclic, and the wrapped cell J_R[0] = [x_{n-1}, x_n] belongs to the
    last block at position n."""
    d = math.exp(-nu)
    nb = -(-n // block)
    blk = lambda p: min(p // block, nb - 1)
    per = bc == "periodic"
    # right-moving contributions by position: J_R[k] at position k (k >= 1), the wrapped cell at n
    posR = [(k, JR[k]) for k in range(1, n)] + ([(n, JR[0])] if per else [])
    R = np.zeros(n)
    L = np.zeros(n)
    for i in range(n):
        b = blk(i)
        for p, j in posR:
            bp = blk(p) if p < n else nb - 1
            if bp == b and p <= i:
                R[i] += d ** (i - p) * j
            elif (per and bp == (b - 1) % nb and bp != b) or (not per and bp == b - 1):
                R[i] += d ** ((i - p) % n) * j
        for k in range(n):
            bk = blk(k)
            if bk == b and k >= i:
                L[i] += d ** (k - i) * JL[k]
            elif (per and bk == (b + 1) % nb and bk != b) or (not per and bk == b + 1):
                L[i] += d ** ((k - i) % n) * JL[k]
    return R, L


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n,block", [(61, 9), (64, 16), (40, 13)])
def test_short_blocks_match_explicit_window_sums(bc, op, n, block):
    """Blocks far shorter than K (nu = 0.3: each neighbour exchange drops a factor of only
    e^{-0.3 block}): the block form is exactly the explicit window sums, and visibly not the global
    operator."""
    nu = 0.3
    dx = _dx(bc, n)
    alpha = nu / dx
    v = _line(n, 5)
    ga, gb = (0.9, -0.6) if bc == "dirichlet" else (0.0, 0.0)
    JL, JR = oracle.line_quad(bc, 6, alpha, dx, v)
    R, L = _windows(bc, n, block, nu, JL, JR)
    d = math.exp(-nu)
    ncell = n if bc == "periodic" else n - 1
    i = np.arange(n)
    first = i < block
    last = i >= (-(-n // block) - 1) * block
    if bc == "periodic":
        ref = {"R": R, "L": L, "0": 0.5 * (R + L)}[op]
    elif op == "R":
        ref = R + first * ga * d ** i
    elif op == "L":
        ref = L + last * gb * d ** (ncell - i)
    else:
        A = ga - 0.5 * L[0]
        B = gb - 0.5 * R[-1]
        ref = 0.5 * (R + L) + first * A * d ** i + last * B * d ** (ncell - i)
    got = oracle.line_invL_nn(bc, op, 6, alpha, dx, v, block, ga, gb)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-14 * scale
    glob = oracle.line_invL(bc, op, 6, alpha, dx, v, ga, gb)
    assert np.abs(glob - got).max() > 1e-3 * scale
    if bc == "dirichlet" and op == "0":
        # the end values hold on the block operators (the other end's term is below e^{-nu (n-1)})
        assert abs(got[0] - ga) < 1e-12 and abs(got[-1] - gb) < 1e-12


@pytest.mark.parametrize("op", ["R", "L"])
@pytest.mark.parametrize("nu", [0.01, 0.05])
def test_one_periodic_block_differs_by_the_further_wraps(op, nu):
    """A single periodic block carries its own end integral once (the periodic choice); the global
    operator sums every wrap, A / (1 - mu): their difference is that series' tail, exactly."""
    n = 50
    dx = 1.0 / n
    alpha = nu / dx
    v = _line(n, 8)
    glob = oracle.line_invL("periodic", op, 6, alpha, dx, v)
    nn = oracle.line_invL_nn("periodic", op, 6, alpha, dx, v, n)
    mu = math.exp(-nu * n)
    d = math.exp(-nu)
    i = np.arange(n)
    if op == "R":
        # NN[0] = A (the sweep is zero at x_0)
        tail = nn[0] * d ** i * mu / (1 - mu)
    else:
        # NN at x_{n-1} = J_L[n-1] + B d; B = the block's own I_L(a)
        B = (nn[-1] - oracle.line_quad("periodic", 6, alpha, dx, v)[0][-1]) / d
        tail = B * d ** (n - i) * mu / (1 - mu)
    assert np.abs(glob - nn - tail).max() <= 1e-13 * np.abs(glob).max()
    assert np.abs(tail).max() > 1e-3 * np.abs(glob).max()
