#!/usr/bin/env python3
"""Benchmark of the successive-convolution hot path on one MI355X.

Headline workload: the 3-D heat equation u_t = lap u on [0, 1]^3, 512^3 points including the
boundaries, homogeneous Dirichlet ends, FP64, sixth-order local quadrature, dt = dx, beta = 1,
dimension-split: one "step" is an x, a y and a z pass, each u <- u - D_0[u] along every line of that
axis (3 one-dimensional operator applications per DOF).  Initial data: 16 seeded Gaussian bumps.
At 1.07 GB per field the working set is four times the 256 MB Infinity Cache.

Prints one JSON line.  ``value`` = DOF x operator applications / s (each pass applies one operator);
``config.paper_metric_dof_per_s`` = DOF / (time per step), the paper's DOF/node/s with one GPU as
the node.  ``roofline`` reports the dominant kernel's algorithmic HBM bytes (16 B per DOF: read the
operand once, write the result once) over its mean launch duration, measured with HIP events that
the library records on the launch stream inside the timed steps; ``per_pass`` and ``step`` give the
same ratio per axis pass (all its launches) and per step.  ``traffic`` is FETCH_SIZE + WRITE_SIZE
from the committed rocprofv3 counter summaries when they were taken on the current kernel sources.
``cpu_baseline`` times the FP64 oracle on a bounded sample of the same workload on the host cores.
``beside`` holds the other workloads measured the same way: the same heat step on the mixed
FP32/FP64 path, the 2-D advection-diffusion step (4096^2), the 1-D line workload replicated to
2^18 lines, the Runge-Kutta steps with partial sums (256^3), the ragged batch, the Hamilton-Jacobi
solver with classical and learned weights, a plain device copy, and the nearest-neighbour block form
of Sec. 3 beside the exact carries.

``--only LEG`` runs one leg (for profiling): heat3d_f64, heat3d_mixed, advdiff2d, line1d, batch, hj,
copy, nn, rk.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "DOF updates/s per L^{-1}/D application on 1 GPU; % HBM roofline; error vs FP64"
HEAT_N = 512
ADV_N = 4096
LINE_N, LINE_LINES = 1024, 1 << 18
RK_N = 256
NFIELDS = 4  # 2-D leg: rotate independent fields (134 MB each) so a pass never re-reads from cache


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2007_03041_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".inc", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summaries (None if stale or absent)."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    k = rec.get("workloads", {}).get(workload, {}).get(kernel)
    return None if not k else k.get("hbm_bytes_per_launch")


# ------------------------------------------------------------------------------------------------
# timing
# ------------------------------------------------------------------------------------------------
def measure(sc, torch, step_fn, steps, warmup, profile_steps=3):
    """Times `steps` calls of step_fn after `warmup` untimed ones.

    A short pass first times every launch of the library (HIP events on the launch stream) for the
    per-kernel breakdown and to find the dominant kernel (largest total time per step).  In the timed
    region only the dominant kernel's launches carry library events, and every step is bracketed by
    a pair of events on the same stream for the per-step minimum and median.  Returns a dict."""
    for _ in range(warmup):
        step_fn()
    torch.cuda.synchronize()
    sc.timing_reset()
    sc.timing_select(None)
    sc.timing_enable(True)
    for _ in range(profile_steps):
        step_fn()
    torch.cuda.synchronize()
    sc.timing_enable(False)
    breakdown = sc.timing_read()
    sc.timing_reset()
    dominant = max(breakdown.items(), key=lambda kv: kv[1][0])[0]
    sc.timing_select([dominant])
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    sc.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        step_fn()
        b.record()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    sc.timing_enable(False)
    live = sc.timing_read()
    sc.timing_reset()
    sc.timing_select(None)
    per_step = sorted(a.elapsed_time(b) for a, b in ev)
    tot, cnt = live[dominant]
    return {
        "total_s": total,
        "ms_per_step": 1e3 * total / steps,
        "step_ms_min": per_step[0],
        "step_ms_median": statistics.median(per_step),
        "dominant": dominant,
        "dominant_mean_ms": tot / cnt,
        "dominant_launches_per_step": cnt / steps,
        "kernel_ms": {k: v[0] / v[1] for k, v in breakdown.items()},
        "kernel_launches_per_step": {k: v[1] / profile_steps for k, v in breakdown.items()},
    }


def frac(bytes_, ms):
    gbs = bytes_ / (ms / 1e3) / 1e9
    return {"GBps": gbs, "frac": gbs / HBM_PEAK_GBS}


# ------------------------------------------------------------------------------------------------
# workloads
# ------------------------------------------------------------------------------------------------
def heat3d(sc, torch, dtype_name, steps, warmup, n=HEAT_N):
    """3-D heat workload, dimension-split; returns the leg's record and the final field."""
    import dataclasses

    from paper_2007_03041_amd import workloads as W

    dx = 1.0 / (n - 1)
    g = sc.Grid((n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), ("dirichlet",) * 3)
    tdt = torch.float64
    if dtype_name == "mixed":
        g = dataclasses.replace(g, dtype=sc.SC_F32_MIXED)
        tdt = torch.float32
    elem = 8 if tdt == torch.float64 else 4
    pde = sc.make_pde(nu_diff=1.0, beta=1.0, dt=dx, order=6, split=True)
    st = sc.TimeStepper(g, pde)
    u = W.bump_field(n, device="cuda").to(tdt)
    m = measure(sc, torch, lambda: st.step(u, 1), steps, warmup)
    dof = n ** 3
    apps = 3
    t_step = m["ms_per_step"] / 1e3
    per_pass = {}
    for axis in "xyz":
        ms = sum(v * m["kernel_launches_per_step"][k] for k, v in m["kernel_ms"].items() if k.endswith("_" + axis))
        per_pass[axis] = dict(ms=ms, **frac(2 * elem * dof, ms))
    rec = {
        "dof_applications_per_s": dof * apps / t_step,
        "paper_metric_dof_per_s": dof / t_step,
        "ms_per_step": m["ms_per_step"],
        "step_ms_min": m["step_ms_min"],
        "step_ms_median": m["step_ms_median"],
        "bytes_per_dof_per_pass": 2 * elem,
        "dominant_kernel": m["dominant"],
        "dominant_mean_ms": m["dominant_mean_ms"],
        "dominant": frac(2 * elem * dof, m["dominant_mean_ms"]),
        "per_pass": per_pass,
        "step": frac(3 * 2 * elem * dof, m["step_ms_median"]),
        "kernel_ms": m["kernel_ms"],
    }
    return rec, m, u


def advdiff2d(sc, torch, steps, warmup, n=ADV_N):
    """2-D linear advection-diffusion u_t + u_x + u_y = lap u, 4096^2 periodic on [0, 2 pi]^2, FP64,
    order 4, dimension-split x then y, dt = dx, beta = 1, 8 seeded Fourier modes: each pass applies
    D_R and D_0 to the same operand (2 applications, 16 B/DOF)."""
    from paper_2007_03041_amd import workloads as W

    L = 2 * math.pi
    g = sc.Grid((n, n), (0.0, 0.0), (L, L))
    pde = sc.make_pde(c=(1.0, 1.0), nu_diff=1.0, beta=1.0, dt=L / n, order=4, split=True)
    st = sc.TimeStepper(g, pde)
    fields = [W.fourier_field(n, n, device="cuda") for _ in range(NFIELDS)]
    it = iter(range(1 << 62))
    m = measure(sc, torch, lambda: st.step(fields[next(it) % NFIELDS], 1), steps, warmup)
    dof = n * n
    t = m["ms_per_step"] / 1e3
    per_pass = {}
    for axis in "xy":
        ms = sum(v * m["kernel_launches_per_step"][k] for k, v in m["kernel_ms"].items() if k.endswith("_" + axis))
        per_pass[axis] = dict(ms=ms, **frac(16 * dof, ms))
    return {
        "workload": "2-D linear advection-diffusion, 4096x4096 periodic on [0,2pi]^2, FP64, order-4 quadrature, "
                    "dimension-split x then y, dt=dx, beta=1, 8 seeded Fourier modes, 4 fields rotated",
        "dof_applications_per_s": dof * 4 / t,
        "dof_passes_per_s": dof * 2 / t,
        "paper_metric_dof_per_s": dof / t,
        "ms_per_step": m["ms_per_step"],
        "step_ms_min": m["step_ms_min"],
        "step_ms_median": m["step_ms_median"],
        "dominant_kernel": m["dominant"],
        "dominant": frac(16 * dof, m["dominant_mean_ms"]),
        "per_pass": per_pass,
        "step": frac(32 * dof, m["step_ms_median"]),
        "kernel_ms": m["kernel_ms"],
    }


def line1d(sc, torch, steps, warmup):
    """The 1-D line workload (periodic [0, 1], N = 1024, alpha = 1024, sin(2 pi x) + 0.05 box-filtered
    noise) replicated to 2^18 independent lines (2.1 GB): one L_0^{-1} and one fused S_3 = D + D^2 + D^3
    per step, each reading the operand once and writing the result once."""
    from paper_2007_03041_amd import workloads as W

    g = sc.Grid((LINE_N, LINE_LINES), (0.0, 0.0), (1.0, 1.0))
    base = torch.from_numpy(W.noisy_sine_line(LINE_N, index=1, lines=64)).to("cuda")
    v = base.repeat(LINE_LINES // 64, 1).contiguous()
    out = torch.empty_like(v)
    res = {"workload": "1-D periodic line N=1024 on [0,1], alpha=1024 (nu=1), order 6, replicated to 2^18 lines, FP64"}
    dof = LINE_N * LINE_LINES
    for name, fn in (("invL_0", lambda: sc.apply_invL(v, g, 0, "0", 6, 1024.0, out=out)),
                     ("S3_0", lambda: sc.apply_D_partial_sum(v, g, 0, "0", 6, 1024.0, 3, 1.0, out=out))):
        m = measure(sc, torch, fn, steps, warmup)
        res[name] = {"ms_min": m["step_ms_min"], "ms_median": m["step_ms_median"],
                     "dof_per_s": dof / (m["step_ms_median"] / 1e3),
                     "kernel": m["dominant"], "kernel_mean_ms": m["dominant_mean_ms"],
                     **frac(16 * dof, m["step_ms_median"])}
    return res


def nn_leg(sc, torch, steps, warmup, n=ADV_N):
    """The nearest-neighbour block form (Sec. 3) beside the exact carries: L_R^{-1} (the advection
    operator, alpha = beta / (c dt) at dt = dx, beta = 1: nu = 1, so K = ceil(ln(1e16)) = 37 points)
    along y of a 4096^2 periodic FP64 field, lines cut into 8 virtual blocks of 512 points (one
    chunk each) that exchange only their block-end integrals.  Timed the same way: the exact
    single-read launch, the exact aggregate + apply launches, and the block form (aggregate,
    nearest-neighbour carries, apply)."""
    from paper_2007_03041_amd import workloads as W

    g = sc.Grid((n, n), (0.0, 0.0), (1.0, 1.0))
    alpha = float(n)  # nu = alpha dx = 1
    v = W.fourier_field(n, n, device="cuda")
    out = torch.empty_like(v)
    block = sc.chunk_points(g, 1)
    dof = n * n
    res = {"workload": f"L_R^{{-1}} along y, {n}x{n} periodic FP64, order 6, nu = 1 (K = 37), "
                       f"virtual blocks of {block} points",
           "block_points": block, "window_K": math.ceil(math.log(1e16))}
    legs = (("exact_single_read", None, "1"), ("exact_two_launch", None, None), ("nn_blocks", block, None))
    prev = os.environ.get("SC_SINGLE")
    try:
        for name, blk, single in legs:
            if single is None:
                os.environ.pop("SC_SINGLE", None)
            else:
                os.environ["SC_SINGLE"] = single
            fn = (lambda: sc.apply_invL(v, g, 1, "R", 6, alpha, out=out)) if blk is None else \
                 (lambda: sc.apply_invL_nn(v, g, 1, "R", 6, alpha, blk, out=out))
            m = measure(sc, torch, fn, steps, warmup)
            res[name] = {"ms_min": m["step_ms_min"], "ms_median": m["step_ms_median"],
                         "kernel_ms": m["kernel_ms"], **frac(16 * dof, m["step_ms_median"])}
    finally:
        if prev is None:
            os.environ.pop("SC_SINGLE", None)
        else:
            os.environ["SC_SINGLE"] = prev
    exact = sc.apply_invL(v, g, 1, "R", 6, alpha)
    nn = sc.apply_invL_nn(v, g, 1, "R", 6, alpha, block)
    res["max_rel_diff_nn_vs_exact"] = ((nn - exact).abs().max() / exact.abs().max()).item()
    return res


def rk_leg(sc, torch, steps, warmup, n=RK_N):
    """3-D linear advection-diffusion u_t + c.grad u = nu lap u, 256^3 periodic on [0, 2 pi]^3,
    order 6, c = (1, 0.5, 0.25), nu = 0.01, beta = 0.35, dt = 1e-3, unsplit: one step of forward
    Euler with D (s = 1) and of the s-stage Runge-Kutta forms with the partial sums S_s (s = 2, 3;
    Sec. 2.5), FP64 and mixed.  Each stage is its partial-sum passes alone (two operators on each of
    three axes); the stage combinations ride in their epilogues."""
    from paper_2007_03041_amd import workloads as W

    res = {"workload": f"3-D advection-diffusion {n}^3 periodic, order 6, c=(1, 0.5, 0.25), nu=0.01, beta=0.35, "
                       "dt=1e-3, unsplit; forward Euler (s=1) and SSP Runge-Kutta with S_s (s=2, 3)"}
    u0 = torch.from_numpy(W.random_field((n, n, n), index=90)).to("cuda")
    for dname, dtype, tdt in (("f64", sc.SC_F64, torch.float64), ("mixed", sc.SC_F32_MIXED, torch.float32)):
        g = sc.Grid((n,) * 3, (0.0,) * 3, (2 * math.pi,) * 3, dtype=dtype)
        for s in (1, 2, 3):
            u = u0.to(tdt)
            st = sc.TimeStepper(g, sc.make_pde(c=(1.0, 0.5, 0.25), nu_diff=0.01, beta=0.35, dt=1e-3, order=6,
                                               stages=s))
            m = measure(sc, torch, lambda: st.step(u, 1), steps, warmup)
            res[f"{dname}_s{s}"] = {"ms_min": m["step_ms_min"], "ms_median": m["step_ms_median"],
                                    "dof_steps_per_s": n ** 3 / (m["step_ms_median"] / 1e3),
                                    "launches_per_step": sum(m["kernel_launches_per_step"].values()),
                                    "kernel_ms": m["kernel_ms"]}
            del u, st
    return res


def copy_leg(torch, nbytes=1 << 30, reps=20):
    """A plain device-to-device copy of 1 GiB (torch copy_): the bandwidth a streaming kernel gets."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        dst.copy_(src)
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in ev)
    med = statistics.median(ts)
    return {"bytes_moved": 2 * nbytes, "ms_min": ts[0], "ms_median": med,
            "GBps_median": 2 * nbytes / (med / 1e3) / 1e9, "GBps_best": 2 * nbytes / (ts[0] / 1e3) / 1e9,
            "frac_of_peak_median": 2 * nbytes / (med / 1e3) / 1e9 / HBM_PEAK_GBS}


def batch_legs(sc, torch, reps=5):
    """The batched workload (4096 independent instances on [0, 1], line lengths U{256..16384},
    beta U(0.5, 2), periodic or Dirichlet, 1/16 of them with 256 lines; L_0^{-1} or D_0 per
    instance), FP64 and mixed: the autotuned, graph-replayed batch against one launch per instance
    through the single-instance entry points."""
    from paper_2007_03041_amd import workloads as W

    items, total, ms, ng = W.batch_instances(dirichlet_values=True)
    v64, gv = W.batch_data(items, total, ms, device="cuda", ngvals=ng)
    out = {"workload": "4096 instances, lengths U{256..16384}, beta U(0.5,2), periodic/Dirichlet, 1/16 2-D "
                       "(256 lines), order 6, L_0^{-1} or D_0", "dof": total}
    for name, dtype, tdt in (("f64", sc.SC_F64, torch.float64), ("mixed_f32", sc.SC_F32_MIXED, torch.float32)):
        v = v64.to(tdt)
        o = torch.empty_like(v)
        plan = sc.BatchPlan(items, dtype=dtype, order=6)
        t0 = time.perf_counter()
        plan.tune(v, out=o, g=gv, reps=2)
        t_tune = time.perf_counter() - t0
        plan.apply(v, out=o, g=gv, use_graph=True)
        ref = plan.apply_per_instance(v, g=gv)
        torch.cuda.synchronize()
        rel = ((o.double() - ref.double()).abs().max() / ref.double().abs().max()).item()
        res = {}
        for mode in ("graph", "per_instance"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                if mode == "graph":
                    plan.apply(v, out=o, g=gv, use_graph=True)
                else:
                    plan.apply_per_instance(v, out=o, g=gv)
            torch.cuda.synchronize()
            res[mode] = (time.perf_counter() - t0) / reps
        elem = 8 if dtype == sc.SC_F64 else 4
        out[name] = {
            "graph_ms": 1e3 * res["graph"],
            "per_instance_ms": 1e3 * res["per_instance"],
            "speedup_vs_per_instance": res["per_instance"] / res["graph"],
            "dof_per_s": total / res["graph"],
            "hbm_frac_algorithmic": 2 * elem * total / res["graph"] / 1e9 / HBM_PEAK_GBS,
            "tune_s": t_tune,
            "shapes": plan.describe()["shapes"],
            "max_rel_diff_vs_per_instance": rel,
        }
        plan.close()
        del v, o, ref
    return out


def hj_legs(sc, torch, n=2048, t_end=1.5, cfl=0.5, nsamples=1_000_000, train_steps=1500, batch=8192):
    """The nonlinear Hamilton-Jacobi workload (u_t + |grad u|^2 / 2 = 0, 2048^2 periodic on
    [0, 2 pi]^2, u0 = sin x + sin y, CFL 1/2 -- the 2-D Lax-Friedrichs bound dt (c/dx + c/dy) <= 1;
    at CFL 1 the wave speed grows after the kinks form at this resolution -- adaptive lagged step,
    to t = 1.5 after the kinks form): the proposer trained on the GPU on 1e6 stencils harvested from
    classical (WENO-Z) runs, then the solver with linear, WENO-Z and learned weights timed side by
    side."""
    L = 2 * math.pi
    x = torch.arange(n, dtype=torch.float64, device="cuda") * (L / n)
    u0 = torch.sin(x)[None, :] + torch.sin(x)[:, None]
    out = {"workload": f"H-J u_t + |grad u|^2/2 = 0, {n}x{n} periodic, u0 = sin x + sin y, CFL {cfl}, "
                       f"beta 1, to t = {t_end}"}
    t0 = time.perf_counter()
    Xs, Ys = [], []
    for T in (0.25, 0.75, 1.25, 1.75):
        s = sc.HJSolver(n, L=L, t_end=T, weights="wenoz", cfl=cfl)
        u = u0.clone()
        s.run_to(u)
        for axis in (0, 1):
            X, Y = s.harvest(u, axis)
            g = torch.Generator(device="cuda")
            g.manual_seed(17 + axis)
            idx = torch.randint(0, X.shape[0], (nsamples // 8,), device="cuda", generator=g)
            Xs.append(X[idx])
            Ys.append(Y[idx])
            del X, Y
        del s, u
    X = torch.cat(Xs).contiguous()
    Y = torch.cat(Ys).contiguous()
    t_harvest = time.perf_counter() - t0
    d = torch.tensor(_linear_weights_from(sc, L, cfl), dtype=torch.float32, device="cuda")
    dev = (Y - d).abs().amax(dim=1)
    rare = torch.topk(dev, max(1, X.shape[0] // 100)).indices  # the 1% furthest from the linear weights
    params = torch.empty(sc.mlp_param_count(), dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    # He initialisation of the proposer (weights), zero biases
    with torch.no_grad():
        params.zero_()
        o = 0
        for (nout, nin) in ((32, 8), (32, 32), (3, 32)):
            scale = math.sqrt((2.0 if nout == 32 else 1.0) / nin)
            params[o:o + nout * nin] = torch.randn(nout * nin, generator=gen, device="cuda") * scale
            o += nout * nin + nout
    tr = sc.MlpTrainer(params, max_batch=batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    first = None
    for k in range(train_steps):
        i1 = torch.randint(0, X.shape[0], (batch // 2,), device="cuda", generator=gen)
        i2 = rare[torch.randint(0, rare.numel(), (batch // 2,), device="cuda", generator=gen)]
        idx = torch.cat([i1, i2])
        loss = tr.step(X[idx].contiguous(), Y[idx].contiguous(), 3e-3 if k < 1000 else 1e-3)
        if k == 0:
            first = loss.item()
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    last = loss.item()
    out["training"] = {"samples": int(X.shape[0]), "oversampled": int(rare.numel()),
                       "max_deviation_from_linear": dev.max().item(), "steps": train_steps,
                       "batch": batch, "loss_first": first, "loss_last": last, "harvest_s": t_harvest,
                       "train_s": t_train}
    results = {}
    for weights in ("linear", "wenoz", "learned"):
        s = sc.HJSolver(n, L=L, t_end=t_end, weights=weights, theta=0.05, cfl=cfl)
        s.mlp = params
        u = u0.clone()
        s.init(u)
        s.step(u, 2)  # warm-up
        u = u0.clone()
        s.init(u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run_to(u)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = s.read_state()
        results[weights] = (u, st, dt)
        out[weights] = {"steps": st["steps"], "t": st["t"], "s_total": dt, "ms_per_step": 1e3 * dt / st["steps"],
                        "paper_metric_dof_per_s": n * n * st["steps"] / dt}
        if weights == "learned":
            out[weights]["fallback_rate"] = st["fallbacks"] / max(st["judged"], 1.0)
            out[weights]["mean_judged_error"] = st["judged_err_sum"] / max(st["judged"], 1.0)
    ref = results["wenoz"][0]
    for weights in ("linear", "learned"):
        out[weights]["max_diff_vs_wenoz_solution"] = (results[weights][0] - ref).abs().max().item()
    return out


def _linear_weights_from(sc, L, cfl):
    """Linear weights d of the 5-point rule at nu = beta / CFL, read back from a harvest of a
    quadratic field, where the classical nonlinear weights equal the linear ones."""
    import torch

    s = sc.HJSolver(16, L=L, weights="wenoz", cfl=cfl)
    x = torch.arange(16, dtype=torch.float64, device="cuda")
    u = (0.01 * x * x)[None, :].repeat(16, 1).contiguous()
    X, Y = s.harvest(u, 0)
    return Y[2 * 8].tolist()


# ------------------------------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of the headline workload
# ------------------------------------------------------------------------------------------------
def host_info():
    info = {"nproc": os.cpu_count(), "machine": platform.machine()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keep = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)", "CPU max MHz")
        info["lscpu"] = {k.strip(): v.strip() for k, v in (l.split(":", 1) for l in out.splitlines() if ":" in l)
                         if k.strip() in keep}
    except Exception as e:  # lscpu missing: say so
        info["lscpu"] = f"unavailable: {e}"
    try:
        info["nproc_cmd"] = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout)
    except Exception:
        pass
    return info


def cpu_baseline(sc, torch, reps=10, warm=3):
    """The FP64 oracle on a bounded sample of the headline workload: the x, y and z passes of one
    heat step (u <- u - D_0 u along one axis, order 6, Dirichlet, alpha = 1/sqrt(dx), dx = 1/511),
    each over 512 full lines of 512 points (a plane of the 512^3 step; about 15 s of CPU work in
    all).  Two builds -- the reference build every test checks (-O2 -ffp-contract=off) and a
    labelled -O3 -march=native timing build -- on one thread and on all threads the process may
    use; `warm` untimed runs,
    then `reps` timed runs, minimum and median.  The GPU applies the same passes to the same sample
    arrays and its error against the oracle is reported."""
    import numpy as np

    import oracle
    from paper_2007_03041_amd import workloads as W

    n, lines = HEAT_N, 512
    dx = 1.0 / (n - 1)
    alpha = 1.0 / math.sqrt(dx)
    # x lines: grid (512, lines); y/z lines: grid (lines, 512) along its second axis (strided lines)
    gx = oracle.make_grid((n, lines), (0.0, 0.0), (1.0, 1.0), ("dirichlet", "dirichlet"))
    gy = oracle.make_grid((lines, n), (0.0, 0.0), (1.0, 1.0), ("dirichlet", "dirichlet"))
    full = W.bump_field(n, device="cuda")                       # the headline's initial data
    vx = full[n // 2, n // 2 - lines // 2:n // 2 + lines // 2, :].cpu().numpy().copy()  # x lines
    vy = full[n // 2, :, n // 2 - lines // 2:n // 2 + lines // 2].cpu().numpy().copy()  # y lines
    vz = full[:, n // 2, n // 2 - lines // 2:n // 2 + lines // 2].cpu().numpy().copy()  # z lines
    del full
    cases = ((gx, 0, vx), (gy, 1, vy), (gy, 1, vz))
    sample_dof_apps = 3 * n * lines

    def run():
        return [oracle.apply_D_partial_sum(g, d, "0", 6, alpha, 1, -1.0, v) for g, d, v in cases]

    threads_all = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    timings = {}
    ref_out = None
    for build in ("reference", "native"):
        oracle.use_build(build)
        for nt in (1, threads_all):
            used = oracle.set_threads(nt)
            for _ in range(warm):
                out = run()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                out = run()
                ts.append(time.perf_counter() - t0)
            if build == "reference" and ref_out is None:
                ref_out = out
            ts.sort()
            timings[f"{build}_{used}t"] = {"threads": used, "s_min": ts[0], "s_median": statistics.median(ts),
                                           "dof_applications_per_s_best": sample_dof_apps / ts[0],
                                           "dof_applications_per_s_median": sample_dof_apps / statistics.median(ts)}
    oracle.use_build("reference")
    # the GPU on the same sample arrays
    err = 0.0
    grids = {0: sc.Grid((n, lines), (0.0, 0.0), (1.0, 1.0), ("dirichlet", "dirichlet")),
             1: sc.Grid((lines, n), (0.0, 0.0), (1.0, 1.0), ("dirichlet", "dirichlet"))}
    for (g, d, v), ref in zip(cases, ref_out):
        got = sc.apply_D_partial_sum(torch.from_numpy(v).to("cuda"), grids[d], d, "0", 6, alpha, 1, -1.0)
        err = max(err, float(np.abs(got.cpu().numpy() - ref).max() / np.abs(v).max()))
    best_all = timings[f"reference_{threads_all}t"] if f"reference_{threads_all}t" in timings else None
    head = best_all or max(timings.values(), key=lambda r: r["threads"])
    return {
        "value": head["dof_applications_per_s_median"],
        "unit": "DOF*applications/s",
        "cores": head["threads"],
        "kind": "oracle",
        "sample": f"x, y and z passes of one 512^3 heat step (D_0, order 6, Dirichlet) over {lines} lines of "
                  f"512 points each ({sample_dof_apps} DOF applications per run), {warm} warm-ups + {reps} runs, "
                  "median; reference build -O2 -ffp-contract=off",
        "timings": timings,
        "builds": {"reference": " ".join(oracle.REFERENCE_FLAGS), "native": " ".join(oracle.NATIVE_FLAGS)},
        "host": host_info(),
        "gpu_max_err_vs_oracle_rel_to_max_v": err,
        "context": "paper: > 1e8 DOF/node/s per whole 2-D time step on 40 Xeon Gold 6148 cores (CPU nodes)",
    }


# ------------------------------------------------------------------------------------------------
# counter ingestion: rocprofv3 --pmc summaries -> profiles/traffic_counters.json
# ------------------------------------------------------------------------------------------------
PASS_ORDER = {"heat3d_f64": ("line_pass_fused_x", "line_pass_fused_y", "line_pass_fused_z"),
              "heat3d_mixed": ("line_pass_fused_x", "line_pass_fused_y", "line_pass_fused_z"),
              "advdiff2d": ("line_pass_fused_x", "line_pass_agg_y", "line_pass_apply_y")}


def _counter_means(path, counter, filt):
    """Per-dispatch values of one counter, in dispatch order, for kernels whose name contains filt."""
    import csv

    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter and filt in r["Kernel_Name"]:
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return rows


def ingest_counters(specs, copy_dir):
    """specs: WORKLOAD=DIR pairs, DIR holding fetch/ and write/ rocprofv3 --pmc runs of
    `bench.py --only WORKLOAD`; copy_dir: fetch/ and write/ runs of `bench.py --calibrate-copy`.
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what each reads per byte of a 1 GiB
    device copy; the library's passes of a step are launched in PASS_ORDER, which names them."""
    def per_byte(counter, sub):
        rows = _counter_means(os.path.join(copy_dir, sub, "run_counter_collection.csv"), counter, "")
        big = [v for _, k, v in rows if "copy" in k.lower() or "elementwise" in k.lower()]
        kib = max(big)  # the 1 GiB copy dispatch: its fetch covers the source, its write the destination
        return kib * 1024.0 / float(1 << 30)

    sf, sw = per_byte("FETCH_SIZE", "cfetch"), per_byte("WRITE_SIZE", "cwrite")
    rec = {"kernel_source_sha": kernel_source_sha(), "copy_scale_fetch": sf, "copy_scale_write": sw,
           "note": "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) divided by what each counter reads per byte "
                   "moved by a 1 GiB device copy, averaged over every dispatch of the pass",
           "commands": ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/cfetch -o run -- python3 bench.py "
                        "--calibrate-copy",
                        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/cwrite -o run -- python3 bench.py "
                        "--calibrate-copy"],
           "workloads": {}}
    for spec in specs:
        wl, d = spec.split("=", 1)
        names = PASS_ORDER[wl]
        out = {}
        for counter, sub, scale, key in (("FETCH_SIZE", "fetch", sf, "fetch_bytes_per_launch"),
                                         ("WRITE_SIZE", "write", sw, "write_bytes_per_launch")):
            rows = _counter_means(os.path.join(d, sub, "run_counter_collection.csv"), counter, "scx::")
            acc = {}
            for i, (_, kname, v) in enumerate(rows):
                nm = names[i % len(names)]
                e = acc.setdefault(nm, {"rocprof_name": kname, "vals": []})
                e["vals"].append(v * 1024.0 / scale)
            for nm, e in acc.items():
                o = out.setdefault(nm, {"rocprof_name": e["rocprof_name"], "dispatches": len(e["vals"])})
                o[key] = sum(e["vals"]) / len(e["vals"])
        for o in out.values():
            o["hbm_bytes_per_launch"] = o.get("fetch_bytes_per_launch", 0.0) + o.get("write_bytes_per_launch", 0.0)
        rec["workloads"][wl] = out
        for sub, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
            rec["commands"].append(f"rocprofv3 --pmc {counter} --output-format csv -d DIR/{sub} -o run -- python3 "
                                   f"bench.py --only {wl} --steps 2 --warmup 1")
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline only (no beside legs)")
    ap.add_argument("--only", choices=("heat3d_f64", "heat3d_mixed", "advdiff2d", "line1d", "batch", "hj", "copy",
                                       "nn", "rk"))
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--ingest-counters", nargs="+", metavar="WORKLOAD=DIR",
                    help="write profiles/traffic_counters.json from rocprofv3 --pmc runs (no GPU needed)")
    ap.add_argument("--copy-dir", help="with --ingest-counters: the copy calibration runs")
    args = ap.parse_args()
    if args.ingest_counters:
        print(json.dumps(ingest_counters(args.ingest_counters, args.copy_dir), indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2007_03041_amd as sc

    if args.calibrate_copy:
        # a plain copy of known size, for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings
        print(json.dumps(copy_leg(torch, reps=5)))
        return
    sc.load()
    if args.only:
        if args.only in ("heat3d_f64", "heat3d_mixed"):
            rec = heat3d(sc, torch, args.only.split("_")[1], args.steps, args.warmup)[0]
        elif args.only == "advdiff2d":
            rec = advdiff2d(sc, torch, args.steps, args.warmup)
        elif args.only == "line1d":
            rec = line1d(sc, torch, args.steps, args.warmup)
        elif args.only == "batch":
            rec = batch_legs(sc, torch)
        elif args.only == "hj":
            rec = hj_legs(sc, torch)
        elif args.only == "nn":
            rec = nn_leg(sc, torch, args.steps, args.warmup)
        elif args.only == "rk":
            rec = rk_leg(sc, torch, args.steps, args.warmup)
        else:
            rec = copy_leg(torch)
        print(json.dumps({"only": args.only, **rec}), flush=True)
        return

    head, m, u64 = heat3d(sc, torch, "f64", args.steps, args.warmup)
    dof = HEAT_N ** 3
    name = m["dominant"]
    alg_bytes = 16 * dof
    achieved = alg_bytes / (m["dominant_mean_ms"] / 1e3) / 1e9
    out = {
        "metric": METRIC,
        "value": head["dof_applications_per_s"],
        "unit": "DOF*applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "3-D heat equation, 512^3 incl. boundaries on [0,1]^3, Dirichlet 0, FP64, order-6 local "
                        "quadrature, dimension-split x, y, z passes of u <- u - D_0 u, dt=dx, beta=1, "
                        "16 seeded Gaussian bumps",
            "grid": [HEAT_N] * 3,
            "operator_applications_per_step": 3,
            "paper_metric_dof_per_s": head["paper_metric_dof_per_s"],
            "step_ms_min": head["step_ms_min"],
            "step_ms_median": head["step_ms_median"],
            "kernel_ms": head["kernel_ms"],
            "kernel_source_sha": kernel_source_sha(),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": name,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": load_traffic("heat3d_f64", name),
            "algorithmic_bytes_per_launch": alg_bytes,
            "mean_launch_ms": m["dominant_mean_ms"],
            "per_pass": head["per_pass"],
            "step": head["step"],
        },
    }
    if not args.no_extra:
        del u64
        torch.cuda.empty_cache()
        beside = {}
        mixed, _, u32 = heat3d(sc, torch, "mixed", args.steps, args.warmup)
        del u32
        # the two paths on the same initial data and number of steps: the mixed path's error
        from paper_2007_03041_amd import workloads as W

        g64 = sc.Grid((HEAT_N,) * 3, (0.0,) * 3, (1.0,) * 3, ("dirichlet",) * 3)
        import dataclasses

        g32 = dataclasses.replace(g64, dtype=sc.SC_F32_MIXED)
        pde = sc.make_pde(nu_diff=1.0, beta=1.0, dt=1.0 / (HEAT_N - 1), order=6, split=True)
        a = W.bump_field(HEAT_N, device="cuda")
        b = a.to(torch.float32)
        sc.TimeStepper(g64, pde).step(a, 5)
        sc.TimeStepper(g32, pde).step(b, 5)
        mixed["max_rel_err_vs_f64_path_5_steps"] = ((b.double() - a).abs().max() / a.abs().max()).item()
        del a, b
        torch.cuda.empty_cache()
        beside["heat3d_512_mixed"] = mixed
        beside["advdiff2d_4096"] = advdiff2d(sc, torch, args.steps, args.warmup)
        torch.cuda.empty_cache()
        beside["line1d_replicated"] = line1d(sc, torch, args.steps, args.warmup)
        torch.cuda.empty_cache()
        beside["runge_kutta_256"] = rk_leg(sc, torch, args.steps, args.warmup)
        torch.cuda.empty_cache()
        beside["device_copy_1GiB"] = copy_leg(torch)
        torch.cuda.empty_cache()
        beside["nn_blocks_4096"] = nn_leg(sc, torch, args.steps, args.warmup)
        torch.cuda.empty_cache()
        beside["batch_4096"] = batch_legs(sc, torch)
        torch.cuda.empty_cache()
        beside["hamilton_jacobi_2048"] = hj_legs(sc, torch)
        out["beside"] = beside
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
