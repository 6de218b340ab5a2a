#!/usr/bin/env python3
"""Benchmark of the successive-convolution hot path on one MI355X.

Workload: 2-D linear advection-diffusion u_t + u_x + u_y = lap u on [0, 2 pi]^2, 4096 x 4096,
periodic, FP64, fourth-order local quadrature, dimension-split x then y, dt = dx, beta = 1; initial
data 8 seeded random Fourier modes (|k| <= 16, amplitudes U(-1, 1)).  One "step" is one time step:
an x pass applying D_R and D_0 to every x line and a y pass applying them to every y line
(4 one-dimensional operator applications per DOF).

Prints one JSON line.  ``value`` = DOF x operator applications / s (the per-application update
rate); ``paper_metric_dof_per_s`` = DOF / (time per step), the paper's DOF/node/s with one GPU as
the node.  ``roofline`` reports the dominant kernel's algorithmic HBM bytes (16 B per DOF: read the
operand, write the result) over its mean duration measured with HIP events recorded by the library
on the launch stream.  ``cpu_baseline`` times the FP64 oracle on a bounded sample on the host cores
and reports the GPU result's error against it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 4096
ORDER = 4
OPS_PER_STEP = 4
BYTES_PER_DOF_PASS = 16
NFIELDS = 4  # rotate independent fields so one pass never re-reads what the last few wrote


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2007_03041_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".inc")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries (None if stale or absent)."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(sc, torch, grid, pde_kw):
    """The FP64 oracle on a bounded sample (2 full-size steps from the benchmark's initial data),
    timed on the host cores; the GPU runs the same 2 steps and its error against the oracle is
    reported relative to max|u|."""
    import numpy as np

    import oracle
    from paper_2007_03041_amd import workloads as W

    steps = 2
    u0 = W.fourier_field(N, N)
    og = oracle.make_grid((N, N), (0.0, 0.0), (2 * math.pi, 2 * math.pi))
    t0 = time.perf_counter()
    ref = oracle.time_step(og, (1.0, 1.0), 1.0, 1.0, pde_kw["dt"], ORDER, steps, u0, split=True)
    t = time.perf_counter() - t0
    u = torch.from_numpy(u0).to("cuda")
    sc.time_step(u, grid, steps, **pde_kw)
    torch.cuda.synchronize()
    err = float(np.abs(u.cpu().numpy() - ref).max() / np.abs(ref).max())
    return {
        "value": N * N * OPS_PER_STEP * steps / t,
        "unit": "DOF*applications/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{steps} full-size time steps of the benchmark workload ({N}x{N}, FP64), "
                  f"{t:.2f} s wall",
        "gpu_max_rel_err_vs_oracle": err,
    }


def heat3d_legs(sc, torch, reps=4):
    """The 3-D heat workload (512^3 with both ends stored, Dirichlet 0, order 6, 5 dimension-split
    steps u <- u - D_0 u along x, y, z, dt = dx, beta = 1, 16 seeded Gaussian bumps) on the FP64 path and on the
    mixed path (FP32 data, compensated FP32 in-wave carries, FP64 cross-chunk carries and boundary
    constants), timed side by side; the mixed result's error is taken against the FP64 GPU result
    (the FP64 path itself matches the oracle to 1e-12 in the parity tests)."""
    import dataclasses

    from paper_2007_03041_amd import workloads as W

    n, steps = 512, 5
    dx = 1.0 / (n - 1)
    g64 = sc.Grid((n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), ("dirichlet",) * 3)
    g32 = dataclasses.replace(g64, dtype=sc.SC_F32_MIXED)
    pde = sc.make_pde(nu_diff=1.0, beta=1.0, dt=dx, order=6, split=True)
    u0 = W.bump_field(n, device="cuda")
    out, res = {}, {}
    for name, g, dt in (("f64", g64, torch.float64), ("mixed_f32", g32, torch.float32)):
        st = sc.TimeStepper(g, pde)
        u = u0.to(dt, copy=True)
        st.step(u, steps)  # warm-up, and the result compared below
        res[name] = u.to(torch.float64)
        work = u0.to(dt, copy=True)
        t, kname, kmean, kt = measure(sc, torch, lambda: st.step(work, steps), reps, profile_steps=1)
        t /= reps * steps
        elem = 8 if dt == torch.float64 else 4
        kbytes = 2 * elem * n ** 3
        out[name] = {
            "dof_applications_per_s": n ** 3 * 3 / t,
            "paper_metric_dof_per_s": n ** 3 / t,
            "ms_per_step": 1e3 * t,
            "bytes_per_dof_per_pass": 2 * elem,
            "dominant_kernel": kname,
            "dominant_kernel_GBps": kbytes / (kmean / 1e3) / 1e9,
            "dominant_kernel_hbm_frac": kbytes / (kmean / 1e3) / 1e9 / HBM_PEAK_GBS,
            "kernel_ms": kt,
        }
        del st, u, work
    d = (res["mixed_f32"] - res["f64"]).abs().max().item()
    out["mixed_f32"]["max_rel_err_vs_f64_path"] = d / res["f64"].abs().max().item()
    out["workload"] = ("3-D heat equation, 512^3 incl. boundaries, Dirichlet 0, order-6 quadrature, 5 "
                       "dimension-split steps, dt=dx, beta=1, 16 seeded Gaussian bumps")
    return out


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
    to t = 1.5 after the kinks form):
    the proposer trained on the GPU on 1e6 stencils harvested from classical (WENO-Z) runs, then the
    solver with linear, WENO-Z and learned weights timed side by side."""
    L = 2 * math.pi
    x = torch.arange(n, dtype=torch.float64, device="cuda") * (L / n)
    u0 = torch.sin(x)[None, :] + torch.sin(x)[:, None]
    out = {"workload": f"H-J u_t + |grad u|^2/2 = 0, {n}x{n} periodic, u0 = sin x + sin y, CFL {cfl}, "
                       f"beta 1, to t = {t_end}"}
    # training data: stencils of classical runs at four times, 1e6 drawn at random
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
    first = last = None
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


def calibrate_copy(torch, nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE readings."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes_each_way": nbytes, "reps": reps}))


def measure(sc, torch, step_fn, steps, profile_steps=10):
    """Times `steps` calls of step_fn.  A short pass first times every launch of the library (HIP
    events on the launch stream) for the per-kernel breakdown and to find the dominant kernel; in
    the measured region only the dominant kernel's launches carry events (each timed launch adds
    two event records to the stream).  Returns (seconds, dominant kernel, its mean launch ms in the
    measured region, {kernel: mean ms} of the breakdown pass)."""
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
    sc.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_fn()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    sc.timing_enable(False)
    live = sc.timing_read()
    sc.timing_reset()
    sc.timing_select(None)
    tot, cnt = live[dominant]
    return t, dominant, tot / cnt, {k: v[0] / v[1] for k, v in breakdown.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the side-by-side 3-D heat legs")
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2007_03041_amd as sc
    from paper_2007_03041_amd import workloads as W

    if args.calibrate_copy:
        calibrate_copy(torch)
        return

    sc.load()
    L = 2 * math.pi
    dx = L / N
    grid = sc.Grid((N, N), (0.0, 0.0), (L, L))
    pde_kw = dict(c=(1.0, 1.0), nu_diff=1.0, beta=1.0, dt=dx, order=ORDER, split=True)
    pde = sc.make_pde(**pde_kw)
    fields = [W.fourier_field(N, N, device="cuda") for _ in range(NFIELDS)]
    stepper = sc.TimeStepper(grid, pde)

    for i in range(args.warmup):
        stepper.step(fields[i % NFIELDS], 1)
    torch.cuda.synchronize()

    it = iter(range(1 << 62))
    t, name, mean_ms, kernel_ms = measure(sc, torch, lambda: stepper.step(fields[next(it) % NFIELDS], 1),
                                          args.steps)

    ms_per_step = 1e3 * t / args.steps
    dof = N * N
    value = dof * OPS_PER_STEP / (t / args.steps)

    # dominant kernel: the one with the largest total time per step; its mean launch time is taken
    # from the events around its launches in the measured region
    avg_s = mean_ms / 1e3
    # one fused or apply launch reads the operand and writes the result over every DOF once;
    # an aggregate-only launch (chunked passes) reads it once and writes per-chunk scalars
    alg_bytes = (8 if "agg" in name else BYTES_PER_DOF_PASS) * dof
    achieved = alg_bytes / avg_s / 1e9
    traffic = load_traffic(name)

    out = {
        "metric": "DOF updates/s per L^{-1}/D application on 1 GPU; % HBM roofline; error vs FP64",
        "value": value,
        "unit": "DOF*applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "2-D linear advection-diffusion, 4096x4096 periodic on [0,2pi]^2, FP64, "
                        "order-4 local quadrature, dimension-split x then y, dt=dx, beta=1, "
                        "8 seeded Fourier modes",
            "grid": [N, N],
            "operator_applications_per_step": OPS_PER_STEP,
            "fields_rotated": NFIELDS,
            "paper_metric_dof_per_s": dof / (t / args.steps),
            "kernel_ms": kernel_ms,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": name,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg_bytes,
            "mean_launch_ms": avg_s * 1e3,
        },
    }
    if not args.no_extra:
        del fields, stepper
        out["beside"] = {"heat3d_512": heat3d_legs(sc, torch)}
        torch.cuda.empty_cache()
        out["beside"]["batch_4096"] = batch_legs(sc, torch)
        torch.cuda.empty_cache()
        out["beside"]["hamilton_jacobi_2048"] = hj_legs(sc, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, torch, grid, pde_kw)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
