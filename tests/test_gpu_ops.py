"""Every opcode on the GPU, one single-operation program each: the forward
value against the correctly rounded result (mpmath), binary64 and
binary32, and the adjoint against the oracle's dual-number derivative.
The measured worst errors are printed (run with -s to see them)."""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from tests import parity
from tests.test_oracle_ops import BINARY, EXACT, UNARY, grid, rounded, ulps
from workloads.tracer import Program

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# worst error allowed against the correctly rounded value (in units in the
# last place of the result's format); operations that IEEE 754 rounds
# correctly must be exact in strict mode
ULP_BOUND = 4.0


def one_op(op, dtype):
    if op in UNARY:
        ins = [("INPUT", 0, 0, 0), (op, 1, 0, -1), ("OUTPUT", 0, 1, 0)]
        return Program(f"op_{op}_{dtype}", dtype, 2, [1], [1], [], ins)
    ins = [("INPUT", 0, 0, 0), ("INPUT", 1, 0, 1), (op, 0, 0, 1), ("OUTPUT", 0, 0, 0)]
    return Program(f"op_{op}_{dtype}", dtype, 2, [2], [1], [], ins)


def inputs_for(op, dtype, n=512):
    x = grid(op, np.random.default_rng(31), n)
    if dtype == "f32":
        # stay inside binary32's range for the operation and its result
        if op == "EXP":
            x = np.clip(x, -80.0, 80.0)
        elif op in ("SIN", "COS", "TAN"):
            x = np.clip(x, -1e4, 1e4)
        elif op in ("SQ", "MUL"):
            x = np.clip(x, -1e15, 1e15)
        x = x.astype(np.float32).astype(np.float64)
    return x


def gpu(path, dtype, xs, strict):
    import paper_2408_09662_amd as xg
    p = xg.Program(path, strict=int(strict))
    t = torch.from_numpy(np.ascontiguousarray(xs)).to(p.torch_dtype).cuda()
    y = p.eval([t])[0].double().cpu().numpy()
    return p, t, y


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op", UNARY + BINARY)
def test_op_value_against_correct_rounding(op, dtype, tmp_path):
    path = tmp_path / "p.xgp"
    one_op(op, dtype).save(path)
    xs = inputs_for(op, dtype)
    strict = op in EXACT
    _, _, y = gpu(path, dtype, xs, strict)
    ref = rounded(op, xs, 53 if dtype == "f64" else 24)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(y[0]), fin), op
    npdt = np.float64 if dtype == "f64" else np.float32
    u = ulps(y[0][fin], ref[fin], npdt)
    worst = float(u.max()) if u.size else 0.0
    print(f"{op} {dtype}: max {worst:.2f} ulp over {int(fin.sum())} points")
    if strict:
        assert worst == 0.0, (op, dtype, worst)
    else:
        assert worst <= ULP_BOUND, (op, dtype, worst, xs[:, fin][:, np.argmax(u)])


@pytest.mark.parametrize("op", UNARY + BINARY)
def test_op_adjoint_against_dual_numbers(op, tmp_path):
    """x_bar = f'(x) * y_bar for one operation, binary64, y_bar = 1."""
    path = tmp_path / "p.xgp"
    one_op(op, "f64").save(path)
    xs = inputs_for(op, "f64")
    if op in ("SIN", "COS", "TAN"):
        xs = xs[:, np.abs(xs[0]) < 10]
    if op == "EXP":
        xs = np.clip(xs, -300, 300)
    _, J = OProg(path).jacobian([xs])
    p, t, _ = gpu(path, "f64", xs, False)
    g = p.eval_adjoint([t], [torch.ones((1, xs.shape[1]), dtype=torch.float64, device="cuda")])[0]
    g = g.cpu().numpy()
    ok = np.isfinite(J[0]).all(axis=0)
    assert np.isfinite(g[:, ok]).all(), op
    e = parity.max_err([g[:, ok]], [J[0][:, ok]])
    print(f"{op} adjoint: max err {e:.2e}")
    assert e <= 1e-13, (op, e)
