"""GPU parity of the reverse-mode adjoint (x_bar = J^T y_bar) against the
oracle's dual-number Jacobians, plus the dot-product identity and central
differences, and the torch.autograd.Function built on it."""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from tests import parity
from workloads import configs, inputs
from workloads.pendulum import pendulum
from workloads.tracer import worked_example

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def xgmod():
    import paper_2408_09662_amd as xg
    return xg


def save(prog, tmp_path, name="p"):
    path = tmp_path / f"{name}.xgp"
    prog.save(path)
    return path


def gpu_adjoint(path, xs, ybars, dtype="f64", fused=False, **opts):
    xg = xgmod()
    p = xg.Program(path, **opts)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    xin = [torch.from_numpy(np.ascontiguousarray(x)).to(tdt).cuda() for x in xs]
    yb = [torch.from_numpy(np.ascontiguousarray(y)).to(tdt).cuda() for y in ybars]
    res = p.eval_adjoint(xin, yb, with_outputs=fused)
    torch.cuda.synchronize()
    if fused:
        g, y = res
        return [t.double().cpu().numpy() for t in g], [t.double().cpu().numpy() for t in y], p
    return [t.double().cpu().numpy() for t in res], None, p


def test_worked_example_gradient(tmp_path):
    path = save(worked_example(), tmp_path)
    x = np.linspace(-3, 3, 130)[None, :]
    yb = np.ones_like(x)
    g, y, _ = gpu_adjoint(path, [x], [yb], fused=True)
    ref = 2 * (np.sin(x) + x) * (np.cos(x) + 1)
    assert np.max(np.abs(g[0] - ref) / np.maximum(np.abs(ref), 1)) <= 1e-14
    assert np.max(np.abs(y[0] - (np.sin(x) + x) ** 2)) <= 1e-13


def test_rdag_gradient_vs_dual(tmp_path):
    prog = configs.program("rdag200")
    path = save(prog, tmp_path)
    n = 517
    x = inputs.uniform(11, 8, n)
    yb = np.random.default_rng(3).normal(size=(4, n))
    g, _, _ = gpu_adjoint(path, [x], [yb])
    _, ref = OProg(path).vjp([x], [yb])
    assert parity.max_err(g, ref) <= parity.TOL_F64


@pytest.mark.parametrize("seg", [0, 300, -1])
def test_pendulum_gradient_vs_dual(tmp_path, seg):
    path = save(pendulum(7), tmp_path)
    n = 700
    x = inputs.pendulum_state(104, 7, n)
    o = OProg(path)
    y = o.evaluate([x], threads=8)[0]
    yb = 2.0 * y  # gradient of ||s'||^2
    opts = {} if seg == 0 else {"adj_seg_ops": seg}
    g, yg, p = gpu_adjoint(path, [x], [yb], fused=True, **opts)
    _, ref = o.vjp([x], [yb], threads=8)
    rep = parity.report(g, ref, parity.TOL_F64)
    assert rep["max"] <= parity.TOL_F64, (rep, p.info(2))
    assert parity.max_err(yg, [y]) <= parity.TOL_F64


def test_pendulum_gradient_only_mode(tmp_path):
    path = save(pendulum(7), tmp_path)
    n = 333
    x = inputs.pendulum_state(9, 7, n)
    o = OProg(path)
    yb = np.random.default_rng(1).normal(size=(14, n))
    g, _, _ = gpu_adjoint(path, [x], [yb], fused=False)
    _, ref = o.vjp([x], [yb], threads=8)
    assert parity.max_err(g, ref) <= parity.TOL_F64


def test_pendulum_fp32_gradient(tmp_path):
    path = save(pendulum(7, dtype="f32"), tmp_path)
    n = 640
    x = inputs.pendulum_state(104, 7, n).astype(np.float32).astype(np.float64)
    o = OProg(path)
    y = o.evaluate([x], threads=8)[0]
    yb = (2.0 * y).astype(np.float32).astype(np.float64)
    g, _, _ = gpu_adjoint(path, [x], [yb], dtype="f32")
    _, ref = o.vjp([x], [yb], threads=8)
    tol = parity.f32_grad_tol(o, [x], [yb])
    e = parity.max_err(g, ref)
    print(f"fp32 gradient: max err {e:.3e}, tolerance {tol:.3e}")
    assert e <= tol, (e, tol)


def test_dot_product_identity(tmp_path):
    """<ybar, J v> (oracle forward tangents) == <J^T ybar, v> (GPU adjoint)."""
    path = save(pendulum(7), tmp_path)
    n = 256
    rng = np.random.default_rng(5)
    x = inputs.pendulum_state(17, 7, n)
    v = rng.normal(size=(1, 14, n))
    yb = rng.normal(size=(14, n))
    _, Jv = OProg(path).jvp([x], v, threads=8)
    g, _, _ = gpu_adjoint(path, [x], [yb])
    lhs = np.sum(yb * Jv[0], axis=0)
    rhs = np.sum(g[0] * v[0], axis=0)
    scale = np.sum(np.abs(yb * Jv[0]), axis=0)
    assert np.max(np.abs(lhs - rhs) / scale) <= 1e-12


def test_central_differences(tmp_path):
    """Sanity check, not a parity gate: central FD with h = 1e-6 in fp64."""
    path = save(pendulum(7), tmp_path)
    n = 256
    x = inputs.pendulum_state(21, 7, n)
    o = OProg(path)
    yb = np.random.default_rng(8).normal(size=(14, n))
    g, _, _ = gpu_adjoint(path, [x], [yb])
    h = 1e-6
    fd = np.zeros((14, n))
    for k in range(14):
        xp = x.copy()
        xm = x.copy()
        xp[k] += h
        xm[k] -= h
        fd[k] = np.sum(yb * (o.evaluate([xp], threads=8)[0] - o.evaluate([xm], threads=8)[0]), axis=0) / (2 * h)
    rel = np.abs(g[0] - fd) / np.maximum(np.abs(fd), np.sqrt(np.mean(fd ** 2, axis=1, keepdims=True)))
    assert rel.max() <= 1e-6


def test_autograd_function(tmp_path):
    xg = xgmod()
    path = save(pendulum(7), tmp_path)
    n = 300
    x = inputs.pendulum_state(31, 7, n)
    p = xg.Program(path)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    y = xg.XgFunction.apply(p, xt)
    loss = (y * y).sum()
    loss.backward()
    o = OProg(path)
    yr = o.evaluate([x], threads=8)[0]
    _, ref = o.vjp([x], [2.0 * yr], threads=8)
    assert parity.max_err([xt.grad.cpu().numpy()], ref) <= parity.TOL_F64
