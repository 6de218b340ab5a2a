"""GPU parity of batched application (sc_batch_*): many independent instances of uneven length,
line count, alpha, boundary, operator and layout (contiguous or interleaved lines) in one launch
per tile shape, against the FP64 oracle instance by instance (FP64 1e-12, mixed 1e-5, normalised as
in the other parity tests), through the plain, graph-replayed, tuned and one-launch-per-instance
paths."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2007_03041_amd import SC_F32_MIXED, SC_F64, BatchPlan, ScError
from paper_2007_03041_amd import workloads as W

pytestmark = pytest.mark.gpu


def small_batch(count=48, seed=7, interleaved=0.0, nmax=20000, lines=(1, 1, 2, 3, 5, 17)):
    """Ragged instances covering every tile shape: n from 7 to nmax (log-uniform), line counts from
    `lines`, nu from 1e-3 to 20, both boundaries, all operators, k = 0 / 1, Dirichlet values on some;
    a share `interleaved` of them with interleaved lines (axis 1)."""
    r = np.random.default_rng(seed)
    items, off, goff = [], 0, 0
    for i in range(count):
        n = int(round(10 ** r.uniform(math.log10(7), math.log10(nmax))))
        nl = int(r.choice(lines))
        bc = "dirichlet" if r.random() < 0.5 else "periodic"
        cells = n if bc == "periodic" else n - 1
        nu = float(10 ** r.uniform(-3, math.log10(20)))
        lo = float(r.uniform(-1, 1))
        hi = lo + float(r.uniform(0.5, 3))
        it = dict(offset=off, n=n, nlines=nl, lo=lo, hi=hi, alpha=nu * cells / (hi - lo), bc=bc,
                  op=["L", "R", "0"][i % 3], k=int(r.integers(0, 2)), scale=float(r.uniform(-2, 2)), g_offset=-1)
        if bc == "dirichlet" and r.random() < 0.5:
            it["g_offset"] = goff
            goff += 2 * nl
        if interleaved > 0 and r.random() < interleaved:
            it["axis"] = 1
        items.append(it)
        off += n * nl + int(r.integers(0, 5))  # gaps between instances
    v = np.random.default_rng(seed + 1).standard_normal(off)
    g = np.random.default_rng(seed + 2).standard_normal(max(goff, 1))
    return items, v, g


def instance_view(it, a):
    """The instance's points as a 2-D array whose axis `d` holds its lines: (nlines, n) rows of
    contiguous lines (d = 0), or (n, nlines) with the lines as columns (interleaved, d = 1)."""
    n, nl, d = it["n"], it["nlines"], it.get("axis", 0)
    flat = a[it["offset"]:it["offset"] + n * nl]
    return (flat.reshape(nl, n) if d == 0 else flat.reshape(n, nl)), d


def oracle_instance(it, v, g):
    n, nl = it["n"], it["nlines"]
    x, d = instance_view(it, v)
    if d == 0:
        og = oracle.make_grid((n, nl), (it["lo"], 0.0), (it["hi"], 1.0), (it["bc"], "periodic"))
    else:
        og = oracle.make_grid((nl, n), (0.0, it["lo"]), (1.0, it["hi"]), ("periodic", it["bc"]))
    gv = g[it["g_offset"]:it["g_offset"] + 2 * nl].reshape(nl, 2) if it["g_offset"] >= 0 else None
    if it["k"] == 0:
        ref = oracle.apply_invL(og, d, it["op"], 6, it["alpha"], x, gv)
        return ref, np.abs(ref).max()
    ref = oracle.apply_D_partial_sum(og, d, it["op"], 6, it["alpha"], 1, it["scale"], x, gv)
    return ref, abs(it["scale"]) * np.abs(x).max()


def check_all(items, v, g, got, tol):
    worst = 0.0
    for i, it in enumerate(items):
        ref, scale = oracle_instance(it, v, g)
        out = instance_view(it, got)[0]
        e = float(np.abs(out - ref).max() / max(scale, 1e-300))
        worst = max(worst, e)
        assert e < tol, (i, it, e)
    return worst


def to_dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)


@pytest.mark.parametrize("dtype,tol", [(SC_F64, 1e-12), (SC_F32_MIXED, 1e-5)])
def test_small_batch_all_paths(gpu_lib, dtype, tol):
    items, v, g = small_batch()
    dt = torch.float64 if dtype == SC_F64 else torch.float32
    plan = BatchPlan(items, dtype=dtype, order=6)
    vd, gd = to_dev(v, dt), to_dev(g, torch.float64)
    host = lambda t: (torch.cuda.synchronize(), t.double().cpu().numpy())[1]
    a = host(plan.apply(vd, g=gd))
    check_all(items, v, g, a, tol)
    b = host(plan.apply(vd, g=gd, use_graph=True))
    check_all(items, v, g, b, tol)
    c = host(plan.apply_per_instance(vd, g=gd))
    check_all(items, v, g, c, tol)
    plan.close()


@pytest.mark.parametrize("dtype,tol", [(SC_F64, 1e-12), (SC_F32_MIXED, 1e-5)])
def test_interleaved_line_instances(gpu_lib, dtype, tol):
    """Instances whose lines are interleaved (the y lines of small 2-D arrays: 1 to 40 lines of 7 to
    3000 points, chunked beyond 256 or 512 points) beside contiguous ones: every path, and the
    tuned plan, against the oracle."""
    items, v, g = small_batch(count=40, seed=31, interleaved=0.6, nmax=3000, lines=(1, 3, 16, 17, 40))
    assert sum(it.get("axis", 0) for it in items) >= 15
    dt = torch.float64 if dtype == SC_F64 else torch.float32
    plan = BatchPlan(items, dtype=dtype, order=6)
    vd, gd = to_dev(v, dt), to_dev(g, torch.float64)
    host = lambda t: (torch.cuda.synchronize(), t.double().cpu().numpy())[1]
    check_all(items, v, g, host(plan.apply(vd, g=gd)), tol)
    check_all(items, v, g, host(plan.apply(vd, g=gd, use_graph=True)), tol)
    check_all(items, v, g, host(plan.apply_per_instance(vd, g=gd)), tol)
    plan.tune(vd, g=gd, reps=1)
    shapes = plan.describe()["shapes"]
    assert {s["axis"] for s in shapes} == {0, 1}
    check_all(items, v, g, host(plan.apply(vd, g=gd, use_graph=True)), tol)
    plan.close()


def test_tuned_plan_matches_oracle(gpu_lib):
    items, v, g = small_batch(count=30, seed=11)
    plan = BatchPlan(items, dtype=SC_F64, order=6)
    vd, gd = to_dev(v, torch.float64), to_dev(g, torch.float64)
    plan.tune(vd, g=gd, reps=1)
    d = plan.describe()
    assert d["launches"] >= 1 and sum(s["instances"] for s in d["shapes"]) == len(items)
    out = plan.apply(vd, g=gd, use_graph=True)
    torch.cuda.synchronize()
    check_all(items, v, g, out.cpu().numpy(), 1e-12)
    # a second plan of the same classes starts from the tuned shapes
    plan2 = BatchPlan(items, dtype=SC_F64, order=6)
    assert plan2.describe()["shapes"] == d["shapes"]
    plan.close()
    plan2.close()


def test_graph_replays_follow_new_data(gpu_lib):
    """Each replay reads the arrays' current contents; eager work runs between replays.  (The
    batch leaves gaps between instances that no path writes, so both outputs start zeroed.)"""
    items, v, g = small_batch(count=20, seed=21)
    plan = BatchPlan(items, dtype=SC_F64, order=6)
    vd, gd = to_dev(v, torch.float64), to_dev(g, torch.float64)
    out = torch.zeros_like(vd)
    for rep in range(6):
        vd.mul_(1.5).add_(0.25 * rep)
        plan.apply(vd, out=out, g=gd, use_graph=True)
        eager = plan.apply(vd, out=torch.zeros_like(vd), g=gd)
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep


def test_invalid_batches_raise(gpu_lib):
    base = dict(offset=0, n=100, nlines=1, lo=0.0, hi=1.0, alpha=50.0, bc="periodic", op="0", k=0)
    for bad in (dict(n=6), dict(k=2), dict(alpha=-1.0), dict(nlines=0), dict(g_offset=0),
                dict(hi=0.0), dict(alpha=1e6)):
        with pytest.raises(ScError):
            BatchPlan([dict(base, **bad)], dtype=SC_F64, order=6)
    plan = BatchPlan([base], dtype=SC_F64, order=6)
    v = torch.zeros(100, dtype=torch.float64, device="cuda")
    with pytest.raises(ScError):
        plan.apply(v, out=v)  # aliasing
    plan.close()


@pytest.mark.parametrize("dtype,tol", [(SC_F64, 1e-12), (SC_F32_MIXED, 1e-5)])
def test_config4_full_batch(gpu_lib, dtype, tol):
    """4096 instances (lengths U{256..16384}, beta U(0.5, 2), both boundaries, 1/16 with 256
    lines): the graph-replayed batch equals the one-launch-per-instance path, and sampled
    instances match the oracle."""
    items, total, ms, ng = W.batch_instances(dirichlet_values=True)
    dt = torch.float64 if dtype == SC_F64 else torch.float32
    v64, gv = W.batch_data(items, total, ms, device="cuda", ngvals=ng)
    vd = v64.to(dt)
    plan = BatchPlan(items, dtype=dtype, order=6)
    a = plan.apply(vd, g=gv, use_graph=True)
    b = plan.apply_per_instance(vd, g=gv)
    torch.cuda.synchronize()
    rel = ((a.double() - b.double()).abs().max() / b.double().abs().max()).item()
    assert rel < (1e-13 if dtype == SC_F64 else 2e-6), rel
    r = np.random.default_rng(4)
    pick = list(r.choice(len(items), 6, replace=False)) + [i for i, it in enumerate(items) if it["nlines"] > 1][:2]
    vh = v64.cpu().numpy()
    gh = gv.cpu().numpy()
    ah = a.double().cpu().numpy()
    check_all([items[i] for i in pick], vh, gh, ah, tol)
    plan.close()
