"""GPU parity of the forward path against the oracle (call through the C ABI).

Sizes span several 64-instance tiles and a ragged tail; the full workload
sizes are checked on sampled instances the oracle evaluates one by one.
"""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from tests import parity
from workloads import configs, inputs
from workloads.mpc import cartpole_mpc
from workloads.pendulum import pendulum
from workloads.rdag import rdag
from workloads.tracer import Program as WProg, worked_example

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def xgmod():
    import paper_2408_09662_amd as xg
    return xg


def oracle_for(prog, tmp_path, name="p"):
    path = tmp_path / f"{name}.xgp"
    prog.save(path)
    return OProg(path), path


def gpu_eval(path_or_prog, xs, dtype, **opts):
    xg = xgmod()
    p = xg.Program(path_or_prog, **opts)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    xin = [torch.from_numpy(np.ascontiguousarray(x)).to(tdt).cuda() for x in xs]
    ys = p.eval(xin)
    torch.cuda.synchronize()
    return [y.double().cpu().numpy() for y in ys], p


def test_worked_example(tmp_path):
    o, path = oracle_for(worked_example(), tmp_path)
    x = np.array([[0.0, 0.5, 1.0, np.pi / 2, np.pi, -2.0, 1e-8, 3.75] * 20])
    ys, _ = gpu_eval(path, [x], "f64")
    rs = o.evaluate([x])
    assert parity.max_err(ys, rs) <= parity.TOL_F64


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000])
def test_rdag_config1(tmp_path, n):
    prog = configs.program("rdag200")
    o, path = oracle_for(prog, tmp_path)
    x = inputs.uniform(101, 8, n)
    ys, _ = gpu_eval(path, [x], "f64")
    assert parity.max_err(ys, o.evaluate([x])) <= parity.TOL_F64


def test_pendulum_fp64_ragged(tmp_path):
    o, path = oracle_for(pendulum(7), tmp_path)
    x = inputs.pendulum_state(102, 7, 4133)
    ys, p = gpu_eval(path, [x], "f64")
    rep = parity.report(ys, o.evaluate([x], threads=8), parity.TOL_F64)
    assert rep["max"] <= parity.TOL_F64, rep


def test_pendulum_fp32_ragged(tmp_path):
    o, path = oracle_for(pendulum(7, dtype="f32"), tmp_path)
    x = inputs.pendulum_state(102, 7, 1537).astype(np.float32).astype(np.float64)
    ys, _ = gpu_eval(path, [x], "f32")
    r64 = o.evaluate([x], 64, threads=8)
    r32 = o.evaluate([x], 32, threads=8)
    e32 = parity.max_err(r32, r64)
    tol = max(parity.TOL_F32, 4 * e32)
    assert parity.max_err(ys, r64) <= tol, (parity.max_err(ys, r64), e32)


def test_pendulum_full_size_sampled(tmp_path):
    n = configs.ITEMS["pend7"].n
    o, path = oracle_for(pendulum(7), tmp_path)
    x = inputs.pendulum_state(102, 7, n)
    ys, _ = gpu_eval(path, [x], "f64")
    idx = np.random.default_rng(0).choice(n, 300, replace=False)
    idx = np.concatenate([idx, [0, n - 1]])
    rs = o.evaluate([x[:, idx]], threads=8)
    assert parity.max_err([ys[0][:, idx]], rs) <= parity.TOL_F64


def test_mpc_fp64(tmp_path):
    o, path = oracle_for(cartpole_mpc(), tmp_path)
    x = inputs.cartpole_state(103, 333)
    ys, p = gpu_eval(path, [x], "f64")
    rep = parity.report(ys, o.evaluate([x], threads=8), parity.TOL_F64_MPC)
    assert rep["max"] <= parity.TOL_F64_MPC, rep
    assert p.info(0)["n_chunks"] > 1


def test_pitch_larger_than_n(tmp_path):
    xg = xgmod()
    o, path = oracle_for(configs.program("rdag200"), tmp_path)
    n = 200
    x = inputs.uniform(7, 8, n)
    big = torch.zeros((8, 256), dtype=torch.float64, device="cuda")
    big[:, :n] = torch.from_numpy(x).cuda()
    out = torch.full((4, 300), float("nan"), dtype=torch.float64, device="cuda")
    p = xg.Program(path)
    p.eval([big[:, :n]], outputs=[out[:, :n]], n=n)
    torch.cuda.synchronize()
    y = out.cpu().numpy()
    assert parity.max_err([y[:, :n]], o.evaluate([x])) <= parity.TOL_F64
    assert np.all(np.isnan(y[:, n:])), "wrote past n"


def test_n_zero_and_errors(tmp_path):
    xg = xgmod()
    _, path = oracle_for(configs.program("rdag200"), tmp_path)
    p = xg.Program(path)
    x = torch.zeros((8, 10), dtype=torch.float64, device="cuda")
    p.eval([x], n=0)  # no-op
    with pytest.raises(xg.XgError, match="dtype"):
        p.eval([x.float()])  # wrong dtype caught by the binding
    buf = torch.zeros((8, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(xg.XgError, match="XG_EALIAS"):
        p.eval([buf], outputs=[buf[:4]])


def _strict_program(seed, n_ops=300):
    """Random program over correctly rounded ops only."""
    rng = np.random.default_rng(seed)
    ins = [("CONST", 0, 0, -1)] + [("INPUT", k + 1, 0, k) for k in range(6)]
    live = list(range(1, 7))
    slot = 7
    for _ in range(n_ops):
        op = rng.choice(["ADD", "SUB", "MUL", "DIV", "SQRT", "NEG", "FABS", "FMIN", "FMAX", "SQ"])
        a = int(rng.choice(live[-20:]))
        b = int(rng.choice(live[-20:]))
        if op == "DIV":
            ins.append(("FABS", slot, b, -1))
            ins.append(("ADD", slot + 1, slot, 0))
            ins.append(("DIV", slot + 2, a, slot + 1))
            slot += 3
        elif op == "SQRT":
            ins.append(("FABS", slot, a, -1))
            ins.append(("SQRT", slot + 1, slot, -1))
            slot += 2
        elif op in ("NEG", "FABS"):
            ins.append((op, slot, a, -1))
            slot += 1
        elif op in ("MUL", "SQ"):
            # squash the operand to (-1, 1) first: a / (1 + |a|)
            ins.append(("FABS", slot, a, -1))
            ins.append(("ADD", slot + 1, slot, 0))
            ins.append(("DIV", slot + 2, a, slot + 1))
            if op == "SQ":
                ins.append(("SQ", slot + 3, slot + 2, -1))
            else:
                ins.append(("MUL", slot + 3, slot + 2, b))
            slot += 4
        else:
            ins.append((op, slot, a, b))
            slot += 1
        live.append(slot - 1)
    ins += [("OUTPUT", 0, live[-1 - k], k) for k in range(4)]
    return WProg("strict", "f64", slot, [6], [4], [1.0], ins)


@pytest.mark.parametrize("seed", [1, 2])
def test_strict_mode_bitwise(tmp_path, seed):
    """Without FMA contraction, correctly rounded ops match the oracle bit for bit."""
    prog = _strict_program(seed)
    o, path = oracle_for(prog, tmp_path)
    x = inputs.uniform(seed, 6, 777)
    ys, _ = gpu_eval(path, [x], "f64", strict=1)
    r = o.evaluate([x])[0]
    assert np.isfinite(r).all()
    same = (ys[0] == r) | (np.isnan(ys[0]) & np.isnan(r))
    assert same.all(), np.flatnonzero(~same)[:10]


@pytest.mark.parametrize("opts", [dict(reg_budget=24), dict(reg_budget=24, lds_slots=4),
                                  dict(chunk_ops=500), dict(ipt=2), dict(block=256, ipt=4)])
def test_plan_variants_agree(tmp_path, opts):
    """Spilling to LDS / global, chunking and instances-per-thread change
    only where values live, never what is computed."""
    o, path = oracle_for(pendulum(7), tmp_path)
    x = inputs.pendulum_state(5, 7, 1111)
    ys, p = gpu_eval(path, [x], "f64", **opts)
    assert parity.max_err(ys, o.evaluate([x], threads=8)) <= parity.TOL_F64, (opts, p.info(0))


def test_mixed_precision_mpc(tmp_path):
    """Dynamics/Jacobians/cost in binary32, KKT LDL^T and update in binary64:
    parity with the oracle's mixed evaluation (same per-instruction
    precision), error against full fp64 stated."""
    from workloads.mpc import cartpole_mpc
    o, path = oracle_for(cartpole_mpc(precision="mixed"), tmp_path, "mixed")
    of, _ = oracle_for(cartpole_mpc(), tmp_path, "full")
    x = inputs.cartpole_state(103, 500)
    ys, _ = gpu_eval(path, [x], "f64")
    rm = o.evaluate([x], threads=8)
    rf = of.evaluate([x], threads=8)
    e_mixed = parity.max_err(rm, rf)  # inherent error of the mixed program
    assert e_mixed <= 1e-5
    tol = max(parity.TOL_F32, 4 * e_mixed)
    assert parity.max_err(ys, rm) <= tol, (parity.max_err(ys, rm), e_mixed)
    assert parity.max_err(ys, rf) <= tol


@pytest.mark.parametrize("key", ["mpc_m1", "mpc_m2", "mpc_m4", "mpc_m5"])
def test_mpc_iteration_sweep(key):
    """The closed-form MPC at M = 1 (real-time iteration), 2, 4 and 5 SQP
    iterations: fp64 parity with the oracle on a ragged instance count."""
    path = configs.program_path(key)
    x = configs.ITEMS[key].make_inputs(700)[0]
    ys, _ = gpu_eval(path, [x], "f64")
    rep = parity.report(ys, OProg(path).evaluate([x], threads=8), parity.TOL_F64_MPC)
    assert rep["max"] <= parity.TOL_F64_MPC, rep


@pytest.mark.parametrize("key,n", [("ldl4", 1000), ("ldl10", 777), ("ldl22", 333),
                                   ("ldl48", 200), ("ldl104", 130)])
def test_ldl_family(key, n):
    """The LDL^T-solve benchmark family, every size, ragged instance counts."""
    path = configs.program_path(key)
    xs = configs.ITEMS[key].make_inputs(n)
    ys, _ = gpu_eval(path, xs, "f64")
    rep = parity.report(ys, OProg(path).evaluate(xs, threads=8), parity.TOL_F64)
    assert rep["max"] <= parity.TOL_F64, rep
