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
  4  a batch of independent instances on [0, 1]: line lengths U{256..16384}, beta U(0.5, 2)
     (alpha = beta / dx), periodic or Dirichlet(0) with probability 1/2 each; 1-D instances with
     probability 15/16, otherwise 256 lines of that length; operator L_0, applied as L^{-1} or D
     with probability 1/2 each; data sin(2 pi m x) (m ~ U{1..8}) plus 0.05 times Gaussian noise
     smoothed by a 9-point box filter over the flat batch array
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


def batch_instances(count: int = 4096, index: int = 4, nmin: int = 256, nmax: int = 16384, p2d: float = 1 / 16,
                    lines2d: int = 256, beta=(0.5, 2.0), p_dirichlet: float = 0.5, ops=("0",),
                    dirichlet_values: bool = False):
    """Workload 4: instance descriptors (dicts for ``BatchPlan``) laid out back to back, the element
    count of the batch arrays, the per-instance wave numbers m, and the number of FP64 Dirichlet
    values (2 per line of every Dirichlet instance when ``dirichlet_values``, else 0)."""
    g = rng(index)
    items, off, goff, ms = [], 0, 0, []
    for _ in range(count):
        n = int(g.integers(nmin, nmax + 1))
        nl = lines2d if g.random() < p2d else 1
        bc = "dirichlet" if g.random() < p_dirichlet else "periodic"
        b = float(g.uniform(*beta))
        cells = n if bc == "periodic" else n - 1
        it = dict(offset=off, n=n, nlines=nl, lo=0.0, hi=1.0, alpha=b * cells, bc=bc,
                  op=ops[int(g.integers(0, len(ops)))], k=int(g.integers(0, 2)), scale=1.0, g_offset=-1)
        if bc == "dirichlet" and dirichlet_values:
            it["g_offset"] = goff
            goff += 2 * nl
        items.append(it)
        ms.append(int(g.integers(1, 9)))
        off += n * nl
    return items, off, ms, goff


def batch_data(items, total: int, ms, index: int = 4, device=None, ngvals: int = 0):
    """Workload 4 data for ``batch_instances``: the flat FP64 batch array (torch tensor on
    ``device``, or numpy when ``device`` is None) and the Dirichlet values (or None)."""
    import torch

    dev = "cpu" if device is None else device
    gen = torch.Generator(device=dev)
    gen.manual_seed(SEED0 + index)
    noise = torch.randn(total + 8, generator=gen, dtype=torch.float64, device=dev)
    c = torch.cumsum(noise, 0)
    box = (c[8:] - torch.cat([torch.zeros(1, dtype=torch.float64, device=dev), c[:-9]])) / 9.0
    lens = torch.tensor([it["n"] * it["nlines"] for it in items], device=dev)
    n_el = torch.repeat_interleave(torch.tensor([it["n"] for it in items], device=dev), lens)
    m_el = torch.repeat_interleave(torch.tensor(ms, dtype=torch.float64, device=dev), lens)
    cells = torch.repeat_interleave(
        torch.tensor([it["n"] if it["bc"] == "periodic" else it["n"] - 1 for it in items], dtype=torch.float64,
                     device=dev), lens)
    start = torch.repeat_interleave(torch.tensor([it["offset"] for it in items], device=dev), lens)
    pos = (torch.arange(total, device=dev) - start) % n_el
    x = pos.to(torch.float64) / cells
    v = torch.sin(2 * math.pi * m_el * x) + 0.05 * box
    gv = None
    if ngvals:
        gv = torch.rand(ngvals, generator=gen, dtype=torch.float64, device=dev) * 2 - 1
    if device is None:
        return v.numpy(), None if gv is None else gv.numpy()
    return v, gv
