"""GPU parity of the nonlinear Hamilton-Jacobi example and of the learned weight proposer against
their oracles (oracle/hj.py, oracle/mlp.py).

* the proposer's forward (matrix cores, BF16 operands, FP32 sums) against the oracle's forward with
  the same operands rounded to BF16 (sums in FP64); its gradients likewise; one Adam step;
* the solver with linear and WENO-Z weights against the oracle's solver (FP64, 1e-10 of max |u|);
* training samples (features, WENO-Z weights) against the oracle's;
* training on stencils harvested from classical runs, then what the trained proposer gains: the
  learned-weight solution after the kinks form is closer to the exact solution than the solution
  with the paper's linear weights, close to the WENO-Z one, with few fallbacks."""
import math

import numpy as np
import pytest
import torch

from oracle import hj, mlp
import paper_2007_03041_amd as sc

pytestmark = pytest.mark.gpu
L = 2 * math.pi


def flat(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"]])


def unflat(v):
    v = np.asarray(v, dtype=float)
    o, out = 0, {}
    for k, shape in (("W1", (32, 8)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)), ("W3", (3, 32)), ("b3", (3,))):
        size = int(np.prod(shape))
        out[k] = v[o:o + size].reshape(shape)
        o += size
    return out


def random_params(seed):
    r = np.random.default_rng(seed)
    p = mlp.init_params(seed)
    for k in p:
        p[k] = p[k] + 0.1 * r.standard_normal(p[k].shape)
    return p


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


# One BF16 ulp is at most 2^-7 of the value it rounds.  The GPU and the oracle round the same
# operands to BF16; they can round one differently only where the GPU's FP32 value and the oracle's
# FP64 value straddle a rounding boundary, and then the two differ by one BF16 ulp.
BF16_ULP = 2.0 ** -7
F32_EPS = 2.0 ** -24


def forward_error_bound(p32, X):
    """Per-element first-order bound on |omega_gpu - omega_oracle| when every BF16-rounded
    activation may differ by one BF16 ulp plus what it inherits, and every FP32 sum of m terms by
    m 2^-24 of its magnitude; the softmax moves omega_k by at most omega_k (|dz_k| + max_j |dz_j|)."""
    r = mlp.bf16
    W1, W2, W3 = (np.abs(r(p32[k])) for k in ("W1", "W2", "W3"))
    om, c = mlp.forward(p32, X, emulate_bf16=True)
    e1 = F32_EPS * 9 * (np.abs(c["x0"]) @ W1.T + np.abs(p32["b1"]))
    eh1 = BF16_ULP * np.maximum(c["z1"], 0.0) + e1
    e2 = eh1 @ W2.T + F32_EPS * 33 * (np.abs(c["h1r"]) @ W2.T + np.abs(p32["b2"]))
    eh2 = BF16_ULP * np.maximum(c["z2"], 0.0) + e2
    e3 = eh2 @ W3.T + F32_EPS * 33 * (np.abs(c["h2r"]) @ W3.T + np.abs(p32["b3"]))
    bound = om * (e3 + e3.max(axis=-1, keepdims=True)) + 8 * F32_EPS * om
    return om, bound


def test_mlp_forward_matches_oracle_with_bf16_operands(gpu_lib):
    p = random_params(1)
    # the oracle sees the FP32 parameters the GPU holds
    p32 = unflat(flat(p).astype(np.float32).astype(np.float64))
    S = np.random.default_rng(2).standard_normal((3000, 5)) * np.logspace(-5, 0, 3000)[:, None]
    X = mlp.features(S).astype(np.float32).astype(np.float64)
    ref, bound = forward_error_bound(p32, X)
    got = sc.mlp_forward(dev32(flat(p32)), dev32(X)).double().cpu().numpy()
    d = np.abs(got - ref)
    # every element within its bound ...
    assert (d <= bound).all(), (d.max(), np.argmax(d - bound))
    # ... and nearly all of them far inside it: the two sides round differently only rarely
    tight = d <= 64 * F32_EPS * np.maximum(ref, 1e-30) + 1e-9
    print(f"forward: max diff {d.max():.2e}, elements off the FP32 level {1 - tight.mean():.4f}")
    assert tight.mean() > 0.97


def test_mlp_gradients_match_oracle(gpu_lib):
    """Every gradient element against the oracle's backward with the same BF16 roundings.  A weight
    gradient element sum_n g[n, j] h[n, i] can differ by what its two operands may differ by -- one
    BF16 ulp of their own rounding plus one per rounding point upstream (at most 4 ulp) -- and the
    FP32 sum; a bias gradient sum_n g[n, j] likewise."""
    p = random_params(3)
    p32 = unflat(flat(p).astype(np.float32).astype(np.float64))
    r = np.random.default_rng(4)
    n = 1000  # several tiles, ragged last tile
    X = mlp.features(r.standard_normal((n, 5))).astype(np.float32).astype(np.float64)
    T = r.dirichlet(np.ones(3), n).astype(np.float32).astype(np.float64)
    om, cache = mlp.forward(p32, X, emulate_bf16=True)
    g, up = mlp.backward(p32, cache, T, emulate_bf16=True, with_upstream=True)
    tr = sc.MlpTrainer(dev32(flat(p32)), max_batch=n)
    grad, loss = tr.gradient(dev32(X), dev32(T))
    torch.cuda.synchronize()
    gg = unflat(grad.double().cpu().numpy())
    assert abs(loss.item() - mlp.loss(om, T)) < 1e-4 * mlp.loss(om, T)
    kappa = 4 * BF16_ULP
    acts = {"W3": cache["h2r"], "W2": cache["h1r"], "W1": cache["x0"]}
    ups = {"W3": up["z3"], "W2": up["z2"], "W1": up["z1"], "b3": up["z3"], "b2": up["z2"], "b1": up["z1"]}
    frac_tight = []
    for k in g:
        if k.startswith("W"):
            mag = np.abs(ups[k]).T @ np.abs(acts[k])
        else:
            mag = np.abs(ups[k]).sum(axis=0)
        bound = (2 * kappa + n * F32_EPS) * mag + 1e-12
        d = np.abs(gg[k] - g[k])
        assert (d <= bound).all(), (k, float((d / bound).max()))
        frac_tight.append(float((d <= 1e-5 * mag + 1e-12).mean()))
        print(f"gradients {k}: max |diff| / magnitude {float((d / (mag + 1e-30)).max()):.2e}")
    # where no BF16 rounding differs (nearly everywhere) the two agree to the FP32 sums
    print("gradients: fraction of elements within 1e-5 of their magnitude:", frac_tight)
    assert min(frac_tight) > 0.99


def test_adam_steps_match_oracle(gpu_lib):
    """Three Adam steps with different gradients (GPU FP32 against the oracle's FP64): parameters
    and both moments after every step, so the moment accumulation and the bias corrections of steps
    2 and 3 are compared, not only the first step's lr sign(g)."""
    p = random_params(5)
    p32 = unflat(flat(p).astype(np.float32).astype(np.float64))
    params = dev32(flat(p32))
    tr = sc.MlpTrainer(params, max_batch=16)
    q = {k: v.copy() for k, v in p32.items()}
    st = {}
    r = np.random.default_rng(6)
    for step, lr in enumerate((1e-3, 3e-3, 2e-3)):
        gv = (r.standard_normal(params.numel()) * np.logspace(-4, 0, params.numel())).astype(np.float32)
        tr.grad.copy_(torch.from_numpy(gv))
        tr.adam(lr)
        mlp.adam_step(q, unflat(gv.astype(np.float64)), st, lr)
        torch.cuda.synchronize()
        got = unflat(params.double().cpu().numpy())
        gm = unflat(tr.m.double().cpu().numpy())
        gvv = unflat(tr.v.double().cpu().numpy())
        for k in q:
            assert np.abs(got[k] - q[k]).max() < 2e-6 * (1 + np.abs(q[k]).max()), (step, k)
            assert np.abs(gm[k] - st["m_" + k]).max() <= 1e-6 * np.abs(st["m_" + k]).max() + 1e-30, (step, k)
            assert np.abs(gvv[k] - st["v_" + k]).max() <= 1e-6 * np.abs(st["v_" + k]).max() + 1e-30, (step, k)
    assert st["t"] == 3 and tr.t == 3


def hj_u0(n):
    x = np.arange(n) * (L / n)
    return np.sin(x)[None, :] + np.sin(x)[:, None]


@pytest.mark.parametrize("weights,T", [("linear", 0.5), ("wenoz", 1.5)])
def test_solver_matches_oracle(gpu_lib, weights, T):
    n = 64
    u0 = hj_u0(n)
    ref, hist = hj.hj_run(u0, L, T, mode=weights)
    s = sc.HJSolver(n, L=L, t_end=T, weights=weights)
    u = torch.from_numpy(u0.copy()).cuda()
    s.run_to(u)
    st = s.read_state()
    assert st["steps"] == len(hist) and abs(st["t"] - T) < 1e-12
    got = u.cpu().numpy()
    assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


def test_example3_matches_oracle(gpu_lib):
    """Example 3 of Sec. 5.1 (H = (1 + u_x + u_y)^2 / 2 with the manufactured source, u0 = 0, T = 0.5,
    linear weights): the GPU solver against the oracle's per-axis adaptive rule, which here takes
    the same steps (the two speeds are equal), to 1e-10."""
    n, T = 64, 0.5
    ref, hist = hj.hj_run_general(np.zeros((n, n)), L, T, kind="ex3", source=hj.example3_source)
    s = sc.HJSolver(n, L=L, t_end=T, weights="linear", hamiltonian="ex3")
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    s.run_to(u)
    st = s.read_state()
    assert st["steps"] == len(hist) and abs(st["t"] - T) < 1e-12
    assert abs(st["c"] - hist[-1][2]) < 1e-10 * hist[-1][2]
    assert np.abs(u.cpu().numpy() - ref).max() < 1e-10 * np.abs(ref).max()


def test_example3_converges_first_order_on_gpu(gpu_lib):
    """Example 3 on the GPU from 128^2 to 1024^2: the error against u = t (sin x + sin y) at T = 0.5
    falls at first order (the explicit Euler step of Sec. 2.5)."""
    T = 0.5
    errs = []
    for n in (128, 256, 512, 1024):
        s = sc.HJSolver(n, L=L, t_end=T, weights="linear", hamiltonian="ex3")
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        s.run_to(u)
        x = torch.arange(n, dtype=torch.float64, device="cuda") * (L / n)
        exact = T * (torch.sin(x)[None, :] + torch.sin(x)[:, None])
        errs.append((u - exact).abs().max().item())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print("Example 3 errors", errs, "rates", rates)
    assert all(r > 0.8 for r in rates[1:]) and 0.9 < rates[-1] < 1.2, rates


def test_harvest_matches_oracle(gpu_lib):
    n = 48
    u0 = hj_u0(n) + 0.3 * np.abs(np.sin(np.arange(n) * (L / n)))[None, :]
    s = sc.HJSolver(n, L=L, weights="wenoz")
    u = torch.from_numpy(u0.copy()).cuda()
    _, _, d, _ = hj.weno5_coefficients(1.0 / 1.0)
    for axis in (0, 1):
        X, Y = s.harvest(u, axis)
        X, Y = X.double().cpu().numpy(), Y.double().cpu().numpy()
        lines = u0 if axis == 0 else u0.T
        SR = np.concatenate([hj.stencils(line, False) for line in lines])
        SL = np.concatenate([hj.stencils(line, True) for line in lines])
        # rows 2p (J_R), 2p + 1 (J_L), points in memory order
        if axis == 1:
            SR = SR.reshape(n, n, 5).transpose(1, 0, 2).reshape(-1, 5)
            SL = SL.reshape(n, n, 5).transpose(1, 0, 2).reshape(-1, 5)
        _, _, dd, _ = hj.weno5_coefficients(1.0)
        assert np.abs(X[0::2] - mlp.features(SR)).max() < 1e-6
        assert np.abs(X[1::2] - mlp.features(SL)).max() < 1e-6
        assert np.abs(Y[0::2] - hj.wenoz_weights(hj.smoothness(SR), dd)).max() < 1e-6
        assert np.abs(Y[1::2] - hj.wenoz_weights(hj.smoothness(SL), dd)).max() < 1e-6


def harvest_classical(n, times, axis_both=True):
    """Stencils of WENO-Z runs at the given times (the classical scheme generates the labels)."""
    Xs, Ys = [], []
    for T in times:
        s = sc.HJSolver(n, L=L, t_end=T, weights="wenoz")
        u = torch.from_numpy(hj_u0(n)).cuda()
        s.run_to(u)
        for axis in (0, 1):
            X, Y = s.harvest(u, axis)
            Xs.append(X)
            Ys.append(Y)
    return torch.cat(Xs), torch.cat(Ys)


def train(X, Y, steps=1500, batch=8192, lr=3e-3, seed=0):
    """Adam on minibatches, half drawn from all samples and half from those whose classical weights
    leave the linear ones (kinks), which are rare."""
    params = dev32(flat(mlp.init_params(seed)))
    tr = sc.MlpTrainer(params, max_batch=batch)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    _, _, d, _ = hj.weno5_coefficients(1.0)
    rare = torch.nonzero((Y - torch.tensor(d, dtype=torch.float32, device="cuda")).abs().amax(dim=1) > 0.1)[:, 0]
    losses = []
    for k in range(steps):
        i1 = torch.randint(0, X.shape[0], (batch // 2,), device="cuda", generator=g)
        i2 = rare[torch.randint(0, rare.numel(), (batch // 2,), device="cuda", generator=g)]
        idx = torch.cat([i1, i2])
        loss = tr.step(X[idx].contiguous(), Y[idx].contiguous(), lr if k < 1000 else lr / 3)
        if k % 100 == 0 or k == steps - 1:
            losses.append(loss.item())
    return params, losses


def test_training_and_what_the_trained_proposer_gains(gpu_lib):
    """Trained on stencils of classical runs at t = 0.25, 0.75, 1.25, 1.75 and judged on those of
    t = 1.5 (held out): on the stencils where the classical nonlinear weights leave the linear ones
    (kinks), the proposal is far closer to them than the linear weights are; in the solver the
    trained proposer falls back rarely (the untrained one always), and the solution after the kinks
    form is no worse than with linear weights and matches the classical one.  (At first order in
    time the nonlinear weights change the solution error by under 1%: the gain is in the weights.)"""
    X, Y = harvest_classical(128, (0.25, 0.75, 1.25, 1.75))
    params, losses = train(X, Y)
    assert losses[-1] < 0.2 * losses[0], losses
    Xh, Yh = harvest_classical(128, (1.5,))
    Ph = sc.mlp_forward(params, Xh)
    _, _, d, _ = hj.weno5_coefficients(1.0)
    dlin = torch.tensor(d, dtype=torch.float32, device="cuda")
    off = (Yh - dlin).abs().amax(dim=1) > 0.1
    assert off.sum().item() > 100
    e_mlp = (Ph - Yh).abs().amax(dim=1)[off].mean().item()
    e_lin = (dlin - Yh).abs().amax(dim=1)[off].mean().item()
    print("held-out kinked stencils:", off.sum().item(), "proposal error", e_mlp, "linear-weight error", e_lin)
    assert e_mlp < 0.5 * e_lin
    n, T = 128, 1.5
    ex = hj.exact_solution(n, n, L, T)
    errs, stats = {}, {}
    for weights in ("linear", "wenoz", "learned"):
        s = sc.HJSolver(n, L=L, t_end=T, weights=weights, theta=0.05)
        s.mlp = params
        u = torch.from_numpy(hj_u0(n)).cuda()
        s.run_to(u)
        errs[weights] = float(np.abs(u.cpu().numpy() - ex).max())
        stats[weights] = s.read_state()
    s0 = sc.HJSolver(n, L=L, t_end=T, weights="learned", theta=0.05)
    s0.mlp = dev32(flat(mlp.init_params(0)))
    u = torch.from_numpy(hj_u0(n)).cuda()
    s0.run_to(u)
    st0 = s0.read_state()
    st = stats["learned"]
    rate = st["fallbacks"] / st["judged"]
    rate0 = st0["fallbacks"] / st0["judged"]
    print("errors", errs, "fallback rate trained", rate, "untrained", rate0)
    assert errs["learned"] <= errs["linear"]
    assert abs(errs["learned"] - errs["wenoz"]) < 0.01 * errs["wenoz"]
    assert rate < 0.2 and rate0 > 0.9


def test_learned_solver_matches_oracle_with_the_same_proposer(gpu_lib):
    """The oracle run with the oracle's proposer (BF16-rounded operands) and the same judge."""
    p = random_params(11)
    p32 = unflat(flat(p).astype(np.float32).astype(np.float64))
    theta = 0.3
    _, _, d, _ = hj.weno5_coefficients(1.0)

    def omega_fn(S):
        om, _ = mlp.forward(p32, mlp.features(S), emulate_bf16=True)
        z = hj.wenoz_weights(hj.smoothness(S), d)
        bad = np.abs(om - z).max(axis=1) > theta
        om[bad] = z[bad]
        return om

    n, T = 32, 0.4
    ref, _ = hj.hj_run(hj_u0(n), L, T, mode="given", omega_fn=omega_fn)
    s = sc.HJSolver(n, L=L, t_end=T, weights="learned", theta=theta)
    s.mlp = dev32(flat(p32))
    u = torch.from_numpy(hj_u0(n)).cuda()
    s.run_to(u)
    assert np.abs(u.cpu().numpy() - ref).max() < 1e-4 * np.abs(ref).max()


@pytest.mark.parametrize("weights", ["linear", "wenoz"])
@pytest.mark.parametrize("shape,steps", [((64, 64), 7), ((300, 200), 10), ((1100, 530), 5), ((2048, 2048), 3)])
def test_fused_step_matches_the_separate_launches(gpu_lib, weights, shape, steps, monkeypatch):
    """The two-pass step (x: w = u - dt Hx; y: u = w - dt Hy, sweeps summed over windows of 64 points
    on either side of each 512-point chunk, nu = 1 here) against the step of separate launches
    (SC_HJ_FUSED=0), both from the same state, odd and even step counts, lines of one and of several
    chunks: the same solution to 1e-12 and the same lagged wave speed and time."""
    n0, n1 = shape
    x = np.arange(n0) * (L / n0)
    y = np.arange(n1) * (L / n1)
    u0 = np.sin(x)[None, :] + np.cos(2 * y)[:, None] + 0.3 * np.sin(x[None, :] + 3 * y[:, None])
    res = {}
    for fused in ("1", "0"):
        monkeypatch.setenv("SC_HJ_FUSED", fused)
        s = sc.HJSolver((n0, n1), L=L, t_end=10.0, weights=weights)
        u = torch.from_numpy(u0.copy()).cuda()
        s.init(u)
        sc.timing_reset()
        sc.timing_select(None)
        sc.timing_enable(True)
        s.step(u, steps)
        sc.timing_enable(False)
        names = set(sc.timing_read())
        assert ("hj_fused_x" in names) == (fused == "1"), names
        res[fused] = (u.cpu().numpy(), s.read_state())
    monkeypatch.delenv("SC_HJ_FUSED")
    (a, sa), (b, sb) = res["1"], res["0"]
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
    assert abs(sa["c"] - sb["c"]) < 1e-12 * sb["c"] and abs(sa["t"] - sb["t"]) < 1e-14 and sa["steps"] == steps


def test_fused_step_not_taken_for_learned_weights_or_example3(gpu_lib):
    for kw in (dict(weights="learned"), dict(weights="linear", hamiltonian="ex3"), dict(weights="linear", cfl=2.0)):
        s = sc.HJSolver(64, L=L, t_end=1.0, **kw)
        if kw.get("weights") == "learned":
            s.mlp = torch.zeros(sc.load().sc_mlp_param_count(), dtype=torch.float32, device="cuda")
        u = torch.from_numpy(hj_u0(64)).cuda()
        s.init(u)
        sc.timing_reset()
        sc.timing_select(None)
        sc.timing_enable(True)
        s.step(u, 2)
        sc.timing_enable(False)
        assert "hj_fused_x" not in set(sc.timing_read()), kw
