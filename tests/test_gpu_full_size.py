"""GPU parity at the workloads' full instance counts, in the launch
configuration the benchmark times (autotuned forward and adjoint plans;
the fused forward+adjoint kernel; the torch.autograd.Function path).
Forward evaluations are checked on every instance against the oracle;
gradients (the oracle's 14-direction dual numbers cost about 30 forward
evaluations each) on sampled instances: a random sample plus the first and
last instance and both sides of the first tile boundary."""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def xgmod():
    import paper_2408_09662_amd as xg
    return xg


def sample(n, k=256, seed=0):
    idx = np.random.default_rng(seed).choice(n, k, replace=False)
    return np.unique(np.concatenate([idx, [0, 63, 64, n - 1]]))


@pytest.mark.parametrize("key,n", [("pend7", 16384), ("pend7", 65536), ("pend7_f32", 16384),
                                   ("mpc", 4096), ("mpc", 65536), ("mpc_m1", 4096), ("mpc_m2", 4096),
                                   ("quad", 10000)])
def test_autotuned_forward_sampled(key, n):
    """Every instance, in the plan the autotuner picks for n (the plan the
    benchmark times: phased cooperative tiles for the pendulum at 16,384,
    the quadcopter step and the one- and two-iteration MPC)."""
    xg = xgmod()
    it = configs.ITEMS[key]
    path = configs.program_path(key)
    xs0 = it.make_inputs(n)
    p = xg.Program(path)
    tdt = p.torch_dtype
    xin = [torch.from_numpy(x).to(tdt).cuda() for x in xs0]
    plan = xg.autotune(p, xin)
    print(f"{key} n={n}: plan {plan}", flush=True)
    y = p.eval(xin)[0].double().cpu().numpy()
    o = OProg(path)
    xs = [x.astype(np.float32).astype(np.float64) for x in xs0] if it.dtype == "f32" else xs0
    ref = o.evaluate(xs, threads=16)  # every instance
    if it.dtype == "f32":
        tol = parity.f32_tol(o, xs)
    else:
        tol = parity.TOL_F64_MPC if key.startswith("mpc") else parity.TOL_F64
    rep = parity.report([y], ref, tol)
    print(f"{key} n={n}: max {rep['max']:.3e} p99 {rep['p99']:.3e} over {rep['over']}", flush=True)
    assert rep["max"] <= tol and rep["over"] == 0, (key, n, rep, p.effective_options())
    assert np.isfinite(y).all()


def test_fused_forward_adjoint_full_size_sampled():
    """The fused kernel the benchmark times at 16,384 instances (seed 2y:
    gradient of the final state's squared norm)."""
    xg = xgmod()
    path = configs.program_path("pend7")
    n = configs.ITEMS["pend7"].n
    x = configs.item_inputs("pend7")[0]
    p = xg.Program(path)
    xin = [torch.from_numpy(x).cuda()]
    xg.autotune(p, xin)
    y = p.eval(xin)[0]
    xg.autotune_adjoint(p, xin, [2.0 * y], fused=True)
    g, y2 = p.eval_adjoint(xin, [2.0 * y], with_outputs=True)
    torch.cuda.synchronize()
    idx = sample(n)
    o = OProg(path)
    yr = o.evaluate([x[:, idx]], threads=8)[0]
    _, gr = o.vjp([x[:, idx]], [2.0 * yr], threads=8)
    assert parity.max_err([g[0].cpu().numpy()[:, idx]], gr) <= parity.TOL_F64
    assert parity.max_err([y2[0].cpu().numpy()[:, idx]], [yr]) <= parity.TOL_F64


@pytest.mark.parametrize("key", ["pend7_grad", "pend7_grad_f32"])
def test_autograd_gradient_full_size_sampled(key):
    """Reverse mode through torch.autograd at 65,536 instances: the gradient
    of the final state's squared norm with respect to the 14 initial
    states, against the oracle's dual-number gradient."""
    xg = xgmod()
    it = configs.ITEMS[key]
    path = configs.program_path(key)
    n = it.n
    x = it.make_inputs(n)[0]
    p = xg.Program(path)
    x0 = torch.from_numpy(x).to(p.torch_dtype).cuda()
    xg.autotune(p, [x0])
    xg.autotune_adjoint(p, [x0], [2.0 * p.eval([x0])[0]], fused=True)
    xt = x0.clone().requires_grad_(True)
    y = xg.XgFunction.apply(p, xt)
    (y * y).sum().backward()
    g = xt.grad.double().cpu().numpy()
    idx = sample(n)
    o = OProg(path)
    if it.dtype == "f64":
        xs = x[:, idx]
        yr = o.evaluate([xs], threads=8)[0]
        _, gr = o.vjp([xs], [2.0 * yr], threads=8)
        assert parity.max_err([g[:, idx]], gr) <= parity.TOL_F64
        assert parity.max_err([y.detach().cpu().numpy()[:, idx]], [yr]) <= parity.TOL_F64
    else:
        xs = x[:, idx].astype(np.float32).astype(np.float64)
        yg = y.detach().double().cpu().numpy()[:, idx]
        yb = (2.0 * yg).astype(np.float32).astype(np.float64)  # the seed the kernel received
        _, gr = o.vjp([xs], [yb], threads=8)
        tol = parity.f32_grad_tol(o, [xs], [yb])
        e = parity.max_err([g[:, idx]], gr)
        print(f"fp32 gradient at {n} instances: max err {e:.3e}, tolerance {tol:.3e}")
        assert e <= tol, (e, tol)
        assert parity.max_err([yg], o.evaluate([xs], threads=8)) <= parity.f32_tol(o, [xs])


@pytest.mark.parametrize("n", [4096, 65536])
def test_autotuned_mixed_precision_mpc_sampled(n):
    """The mixed-precision MPC (binary32 dynamics and cost, binary64 KKT) as
    the benchmark runs it, against the oracle's evaluation of the same
    per-instruction precisions, within max(1e-5, 4 x) the mixed program's
    own error against full fp64."""
    xg = xgmod()
    path = configs.program_path("mpc_mixed")
    x = configs.ITEMS["mpc"].make_inputs(n)[0]
    p = xg.Program(path)
    xin = [torch.from_numpy(x).cuda()]
    xg.autotune(p, xin)
    y = p.eval(xin)[0].cpu().numpy()
    rm = OProg(path).evaluate([x], threads=16)  # every instance
    rf = OProg(configs.program_path("mpc")).evaluate([x], threads=16)
    e_mixed = parity.max_err(rm, rf)
    tol = max(parity.TOL_F32, 4 * e_mixed)
    assert parity.max_err([y], rm) <= tol, (parity.max_err([y], rm), e_mixed)



def test_autotuned_rollout_full_size():
    """The quadcopter rollout as the benchmark runs it: 10,000 environments,
    the autotuned step plan, 20 steps captured in one HIP graph, against the
    oracle's own 20-step rollout (per step within 1e-12; the closed loop is
    contracting, so the composed steps stay within 1e-11)."""
    xg = xgmod()
    path = configs.program_path("quad")
    n, steps = 10000, 20
    z, th = configs.ITEMS["quad"].make_inputs(n)
    p = xg.Program(path)
    tz = torch.from_numpy(z).cuda()
    tth = torch.from_numpy(th).cuda()
    plan = xg.autotune(p, [tz, tth])
    print(f"quad n={n}: plan {plan}", flush=True)
    s = torch.cuda.Stream()
    s0, s1 = tz.clone(), torch.empty_like(tz)
    with torch.cuda.stream(s):
        g = xg.capture_rollout(p, s0, s1, [tth], steps, stream=s)
        g.launch(stream=s)
        s.synchronize()
    fin = (s0 if steps % 2 == 0 else s1).cpu().numpy()
    o = OProg(path)
    r = z.copy()
    for _ in range(steps):
        r = o.evaluate([r, th], threads=16)[0]
    rep = parity.report([fin], [r], 10 * parity.TOL_F64)
    assert rep["max"] <= 10 * parity.TOL_F64, rep
