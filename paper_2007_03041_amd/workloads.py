"""Seeded synthetic inputs with the shapes of the paper's workloads.

Inputs only: nothing here evaluates the method.  Every generator draws its random parameters from
``numpy.random.default_rng(200703041 + index)`` and can return a numpy array (small sizes, for the
oracle) or build the field directly in a torch tensor on a device (large sizes).

  1  1-D periodic line on [0, 1]: sin(2 pi x) + 0.05 * (Gaussian noise smoothed by a circular
     9-point box filter)
  2  2-D periodic field on [0, 2 pi]^2: sum of 8 Fourier modes cos(k.x + phi) with integer wave
     vectors 1 <= max(|kx|, |ky|) <= 16 drawn without replacement, amplitudes U(-1, 1),
     phases U(0, 2 pi)
  3  3-D field on [0, 1]^3 with both ends stored (Dirichlet axes): 16 Gaussian bumps,
     sigma ~ U(0.02, 0.1), centres ~ U(0.25, 0.75)^3, amplitudes ~ U(0.5, 1); the boundary faces are
     set to 0 so the data agree with homogeneous Dirichlet values
"""
from __future__ import annotations

import math

import numpy as np

SEED0 = 200703041


def rng(index: int) -> np.random.Generator:
    return np.random.default_rng(SEED0 + index)


def noisy_sine_line(n: int = 1024, index: int = 1, lines: int = 1) -> np.ndarray:
    """Workload 1 (``lines`` independent draws stacked as rows)."""
    g = rng(index)
    x = np.arange(n) / n
    out = np.empty((lines, n))
    for r in range(lines):
        eta = g.standard_normal(n)
        box = sum(np.roll(eta, j) for j in range(-4, 5)) / 9.0
        out[r] = np.sin(2 * np.pi * x) + 0.05 * box
    return out[0] if lines == 1 else out


def fourier_modes(nmodes: int = 8, kmax: int = 16, index: int = 2):
    g = rng(index)
    cand = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
            if max(abs(kx), abs(ky)) >= 1]
    pick = g.choice(len(cand), size=nmodes, replace=False)
    ks = [cand[i] for i in pick]
    amp = g.uniform(-1.0, 1.0, nmodes)
    phase = g.uniform(0.0, 2 * np.pi, nmodes)
    return ks, amp, phase


def fourier_field(n0: int, n1: int, index: int = 2, device=None):
    """Workload 2 on an n1 x n0 periodic grid of [0, 2 pi]^2 (shape (n1, n0), x contiguous)."""
    ks, amp, phase = fourier_modes(index=index)
    if device is None:
        x = np.arange(n0) * (2 * np.pi / n0)
        y = np.arange(n1) * (2 * np.pi / n1)
        out = np.zeros((n1, n0))
        for (kx, ky), a, ph in zip(ks, amp, phase):
            out += a * np.cos(kx * x[None, :] + ky * y[:, None] + ph)
        return out
    import torch

    x = torch.arange(n0, dtype=torch.float64, device=device) * (2 * math.pi / n0)
    y = torch.arange(n1, dtype=torch.float64, device=device) * (2 * math.pi / n1)
    out = torch.zeros((n1, n0), dtype=torch.float64, device=device)
    for (kx, ky), a, ph in zip(ks, amp, phase):
        out += float(a) * torch.cos(kx * x[None, :] + ky * y[:, None] + float(ph))
    return out


def gaussian_bumps(nbumps: int = 16, index: int = 3):
    g = rng(index)
    sigma = g.uniform(0.02, 0.1, nbumps)
    centre = g.uniform(0.25, 0.75, (nbumps, 3))
    amp = g.uniform(0.5, 1.0, nbumps)
    return sigma, centre, amp


def bump_field(n: int, index: int = 3, device=None, dtype=None):
    """Workload 3 on an n^3 grid of [0, 1]^3 with both ends stored (shape (n, n, n))."""
    sigma, centre, amp = gaussian_bumps(index=index)
    if device is None:
        x = np.linspace(0.0, 1.0, n)
        out = np.zeros((n, n, n))
        for s, c, a in zip(sigma, centre, amp):
            gx = np.exp(-(x - c[0]) ** 2 / (2 * s * s))
            gy = np.exp(-(x - c[1]) ** 2 / (2 * s * s))
            gz = np.exp(-(x - c[2]) ** 2 / (2 * s * s))
            out += a * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
        out[0], out[-1] = 0.0, 0.0
        out[:, 0], out[:, -1] = 0.0, 0.0
        out[:, :, 0], out[:, :, -1] = 0.0, 0.0
        return out
    import torch

    x = torch.linspace(0.0, 1.0, n, dtype=torch.float64, device=device)
    out = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    for s, c, a in zip(sigma, centre, amp):
        gx = torch.exp(-(x - float(c[0])) ** 2 / (2 * s * s))
        gy = torch.exp(-(x - float(c[1])) ** 2 / (2 * s * s))
        gz = torch.exp(-(x - float(c[2])) ** 2 / (2 * s * s))
        out += float(a) * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    out[0], out[-1] = 0.0, 0.0
    out[:, 0], out[:, -1] = 0.0, 0.0
    out[:, :, 0], out[:, :, -1] = 0.0, 0.0
    return out if dtype is None else out.to(dtype)


def random_field(shape, index: int = 11, seed_offset: int = 0) -> np.ndarray:
    """Smooth-plus-noise test data of any shape (parity cases)."""
    g = rng(index + seed_offset)
    a = g.standard_normal(shape)
    grids = np.meshgrid(*[np.arange(s) / s for s in shape], indexing="ij")
    smooth = sum(np.sin(2 * np.pi * (j + 1) * gr + j) for j, gr in enumerate(grids))
    return smooth + 0.1 * a
