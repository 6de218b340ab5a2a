"""sc_apply_invL_noalloc (the entry point for callers that cannot allocate) against sc_apply_invL:
the same kernels on the same inputs, so the results must agree bit for bit.  Each case makes two
calls in a row through the C ABI, the second with a smaller input, so the second runs on scratch
the first left behind."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2007_03041_amd as sc
from paper_2007_03041_amd import Grid
from paper_2007_03041_amd import workloads as W

pytestmark = pytest.mark.gpu


def _pair(gpu_lib, shape_n, bc, dim, op, order, nu, seed, with_g):
    g = Grid(shape_n, tuple(0.0 for _ in shape_n), tuple(1.0 for _ in shape_n), tuple(bc for _ in shape_n))
    v = torch.from_numpy(W.random_field(g.shape, index=seed)).to("cuda")
    lines = v.numel() // int(shape_n[dim])
    gv = None
    if with_g and bc == "dirichlet":
        gv = torch.from_numpy(np.random.default_rng(seed).uniform(-1, 1, 2 * lines)).to("cuda")
    alpha = nu / g.dx(dim)
    ref = sc.apply_invL(v, g, dim, op, order, alpha, g=gv)
    out = torch.full_like(v, float("nan"))
    lib = sc.load()
    gc = g.c()
    rc = lib.sc_apply_invL_noalloc(ctypes.byref(gc), dim, sc.OPS[op], order, alpha,
                                   None if gv is None else gv.data_ptr(), v.data_ptr(), out.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
    assert rc == sc.SC_OK, lib.sc_last_error().decode()
    torch.cuda.synchronize()
    return out, ref


def _needs_scratch(shape_n, dim):
    g = Grid(shape_n)
    return sc.workspace_bytes(g, dim, 0) > 256


@pytest.mark.parametrize("first,second", [
    # y lines of 6 chunks (carries formed in the apply launch), then 3 chunks with Dirichlet values
    (((300, 3000), "periodic", 1, "0", 6, 0.3, 1, False), ((100, 1500), "dirichlet", 1, "R", 6, 0.05, 2, True)),
    # x lines of 19 chunks (the carry launch), then 5 chunks
    (((150000, 2), "periodic", 0, "0", 4, 0.02, 3, False), ((40000, 3), "dirichlet", 0, "L", 6, 0.7, 4, True)),
    # z lines of a 3-D grid, then a shorter x pass
    (((33, 20, 2100), "dirichlet", 2, "0", 6, 0.04, 5, True), ((9000, 2), "periodic", 0, "R", 4, 1.0, 6, False)),
])
def test_noalloc_matches_workspace_entry_point(gpu_lib, first, second):
    for case in (first, second):
        assert _needs_scratch(case[0], case[2]), case
        out, ref = _pair(gpu_lib, *case)
        assert torch.equal(out, ref), (case, (out - ref).abs().max().item())


def test_noalloc_single_tile_and_limit(gpu_lib):
    # a pass that needs no scratch at all
    out, ref = _pair(gpu_lib, (1024, 7), "periodic", 0, "0", 6, 1.0, 7, False)
    assert torch.equal(out, ref)
    # a pass whose chunk totals exceed the fixed scratch is refused before anything is enqueued
    g = Grid((16384, 16384))
    gc = g.c()
    lib = sc.load()
    assert sc.workspace_bytes(g, 1, 0) - 256 > sc.NOALLOC_SCRATCH_BYTES
    rc = lib.sc_apply_invL_noalloc(ctypes.byref(gc), 1, 2, 6, 100.0, None, 0x1000, 0x100000000000, None)
    assert rc == sc.SC_ERR_WORKSPACE
    assert "scratch" in lib.sc_last_error().decode()
