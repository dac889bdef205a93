"""Pins of the oracle's opcode semantics, slot semantics and derivatives.

Each opcode is compared with mpmath (50 digits): the correctly rounded ops
(+, -, *, /, sqrt, neg, fabs, sq, fmin, fmax, comparisons) must match the
correctly rounded reference exactly, in float and in double; the libm ops
within a few ulp.  The worked example of the paper's Fig. 2 (generated
kernel listing: slot 1 reused in place twice) is checked against the stored
mpmath values in tests/golden/worked_example.txt.  Dual-number derivatives
are checked against mpmath derivatives of each op.
"""

import math
import os

import mpmath
import numpy as np
import pytest

from oracle.pyoracle import OracleError, Program as OProg
from workloads.tracer import Program, worked_example

GOLD = os.path.join(os.path.dirname(__file__), "golden")

UNARY = ["NEG", "SQ", "SQRT", "EXP", "LOG", "SIN", "COS", "TAN", "TANH", "ATAN", "FABS"]
BINARY = ["ADD", "SUB", "MUL", "DIV", "FMIN", "FMAX", "LT", "LE", "POW", "ATAN2"]
EXACT = {"NEG", "SQ", "SQRT", "FABS", "ADD", "SUB", "MUL", "DIV", "FMIN", "FMAX", "LT", "LE"}


def one_op_program(op):
    if op in UNARY:
        ins = [("INPUT", 0, 0, 0), (op, 1, 0, -1), ("OUTPUT", 0, 1, 0)]
        return Program(f"op_{op}", "f64", 2, [1], [1], [], ins)
    ins = [("INPUT", 0, 0, 0), ("INPUT", 1, 0, 1), (op, 0, 0, 1), ("OUTPUT", 0, 0, 0)]
    return Program(f"op_{op}", "f64", 2, [2], [1], [], ins)


def grid(op, rng, n=400):
    if op in ("SQRT", "LOG"):
        x = np.exp(rng.uniform(-20, 20, n))
    elif op == "EXP":
        x = rng.uniform(-700, 700, n)
    elif op in ("SIN", "COS", "TAN"):
        x = np.concatenate([rng.uniform(-10, 10, n // 2), rng.uniform(-1e5, 1e5, n - n // 2)])
    else:
        x = rng.uniform(-4, 4, n) * np.exp(rng.uniform(-5, 5, n))
    if op in BINARY:
        y = rng.uniform(-4, 4, n) * np.exp(rng.uniform(-5, 5, n))
        if op == "POW":
            x = np.abs(x) + 1e-3
            y = rng.uniform(-8, 8, n)
        # include exact ties for min/max/comparisons
        if op != "POW":
            y[:20] = x[:20]
        return np.stack([x, y])
    return x[None, :]


def mp_ref(op, a, b=None):
    m = mpmath
    f = {
        "NEG": lambda: -a, "SQ": lambda: a * a, "SQRT": lambda: m.sqrt(a), "EXP": lambda: m.exp(a),
        "LOG": lambda: m.log(a), "SIN": lambda: m.sin(a), "COS": lambda: m.cos(a),
        "TAN": lambda: m.tan(a), "TANH": lambda: m.tanh(a), "ATAN": lambda: m.atan(a),
        "FABS": lambda: abs(a), "ADD": lambda: a + b, "SUB": lambda: a - b, "MUL": lambda: a * b,
        "DIV": lambda: a / b, "FMIN": lambda: min(a, b), "FMAX": lambda: max(a, b),
        "LT": lambda: m.mpf(1 if a < b else 0), "LE": lambda: m.mpf(1 if a <= b else 0),
        "POW": lambda: m.power(a, b), "ATAN2": lambda: m.atan2(a, b),
    }[op]
    return f()


def rounded(op, xs, bits):
    """Reference rounded to `bits` (53 or 24): exact ops computed at that
    precision (mpmath rounds each basic operation correctly); others at
    50 digits and then rounded."""
    out = np.empty(xs.shape[1])
    for i in range(xs.shape[1]):
        if op in EXACT:
            with mpmath.workprec(bits):
                a = mpmath.mpf(float(xs[0, i]))
                b = mpmath.mpf(float(xs[1, i])) if xs.shape[0] > 1 else None
                out[i] = float(mp_ref(op, a, b))
        else:
            with mpmath.workdps(50):
                a = mpmath.mpf(float(xs[0, i]))
                b = mpmath.mpf(float(xs[1, i])) if xs.shape[0] > 1 else None
                v = mp_ref(op, a, b)
            with mpmath.workprec(bits):
                out[i] = float(+v)
    return out


def ulps(y, r, dtype):
    y = y.astype(dtype)
    r = r.astype(dtype)
    sp = np.spacing(np.maximum(np.abs(r), np.finfo(dtype).tiny).astype(dtype))
    with np.errstate(invalid="ignore"):
        d = np.abs(y.astype(np.float64) - r.astype(np.float64)) / sp.astype(np.float64)
    return np.where(y == r, 0.0, d)


@pytest.mark.parametrize("op", UNARY + BINARY)
def test_op_semantics(op, tmp_path):
    prog = one_op_program(op)
    path = tmp_path / "p.xgp"
    prog.save(path)
    o = OProg(path)
    rng = np.random.default_rng(7)
    x = grid(op, rng)
    if op == "EXP":
        x = np.clip(x, -700, 700)
    # double
    y = o.evaluate([x], 64)[0][0]
    r = rounded(op, x, 53)
    if op in EXACT:
        assert np.array_equal(y, r), (op, np.flatnonzero(y != r)[:5])
    else:
        assert ulps(y, r, np.float64).max() <= 2.0, op
    # float: inputs rounded once to float32
    x32 = x.astype(np.float32).astype(np.float64)
    if op == "EXP":
        x32 = np.clip(x32, -80, 80)
    ok = np.all(np.isfinite(x32), axis=0)
    x32 = x32[:, ok]
    y32 = o.evaluate([x32], 32)[0][0]
    r32 = rounded(op, x32, 24)
    fin = np.isfinite(r32) & (np.abs(r32) < 3e38) & (np.abs(r32) > 1e-37)
    if op in EXACT:
        assert np.array_equal(y32[fin], r32[fin]), op
    else:
        assert ulps(y32[fin], r32[fin], np.float32).max() <= 2.0, op


def test_worked_example_golden(tmp_path):
    """Fig. 2 / generated-kernel listing: f(x) = (sin x + x)^2 with slot 1
    written from itself twice (read-all-operands-then-write semantics)."""
    rows = [l.split() for l in open(os.path.join(GOLD, "worked_example.txt")) if not l.startswith("#")]
    x = np.array([[float.fromhex(r[0]) for r in rows]])
    ref = np.array([float(mpmath.mpf(r[1])) for r in rows])
    p = tmp_path / "w.xgp"
    worked_example().save(p)
    y = OProg(p).evaluate([x], 64)[0][0]
    rel = np.abs(y - ref) / np.maximum(np.abs(ref), 1e-300)
    assert rel.max() <= 4 * 2.0 ** -52
    assert y[0] == 0.0
    # If the in-place ADD read its output slot after writing (wrong order),
    # slot 1 would hold 2 sin x or similar: the values above exclude that.


DERIV = {
    "SQ": lambda a, b: (2 * a, None), "SQRT": lambda a, b: (1 / (2 * mpmath.sqrt(a)), None),
    "EXP": lambda a, b: (mpmath.exp(a), None), "LOG": lambda a, b: (1 / a, None),
    "SIN": lambda a, b: (mpmath.cos(a), None), "COS": lambda a, b: (-mpmath.sin(a), None),
    "TAN": lambda a, b: (1 / mpmath.cos(a) ** 2, None), "TANH": lambda a, b: (1 / mpmath.cosh(a) ** 2, None),
    "ATAN": lambda a, b: (1 / (1 + a * a), None), "NEG": lambda a, b: (-1, None),
    "FABS": lambda a, b: (mpmath.sign(a), None),
    "ADD": lambda a, b: (1, 1), "SUB": lambda a, b: (1, -1), "MUL": lambda a, b: (b, a),
    "DIV": lambda a, b: (1 / b, -a / b ** 2),
    "FMIN": lambda a, b: (1, 0) if a <= b else (0, 1), "FMAX": lambda a, b: (1, 0) if a >= b else (0, 1),
    "LT": lambda a, b: (0, 0), "LE": lambda a, b: (0, 0),
    "POW": lambda a, b: (b * mpmath.power(a, b - 1), mpmath.log(a) * mpmath.power(a, b)),
    "ATAN2": lambda a, b: (b / (a * a + b * b), -a / (a * a + b * b)),
}


@pytest.mark.parametrize("op", UNARY + BINARY)
def test_dual_derivatives(op, tmp_path):
    prog = one_op_program(op)
    p = tmp_path / "d.xgp"
    prog.save(p)
    o = OProg(p)
    rng = np.random.default_rng(11)
    x = grid(op, rng, 120)
    if op == "EXP":
        x = np.clip(x, -300, 300)
    if op in ("SIN", "COS", "TAN"):
        x = x[:, np.abs(x[0]) < 10]
    n = x.shape[1]
    k = x.shape[0]
    _, J = o.jacobian([x])
    assert J.shape == (1, k, n)
    for i in range(n):
        with mpmath.workdps(40):
            a = mpmath.mpf(float(x[0, i]))
            b = mpmath.mpf(float(x[1, i])) if k > 1 else None
            da, db = DERIV[op](a, b)
            refs = [da] + ([db] if k > 1 else [])
        for j, r in enumerate(refs):
            r = float(r)
            got = J[0, j, i]
            # 1 - tanh^2 cancels for large |x|: absolute error of a few eps
            atol = 4 * 2.0 ** -52 if op == "TANH" else 1e-300
            assert abs(got - r) <= 1e-13 * abs(r) + atol, (op, j, float(x[0, i]), got, r)


@pytest.mark.parametrize("op", UNARY + BINARY)
def test_dual_derivatives_binary32(op, tmp_path):
    """The binary32 dual numbers: values bitwise those of the binary32
    interpreter, derivatives within a few binary32 roundings of the exact
    derivative at the binary32-rounded point."""
    prog = one_op_program(op)
    p = tmp_path / "d.xgp"
    prog.save(p)
    o = OProg(p)
    rng = np.random.default_rng(12)
    x = grid(op, rng, 120)
    if op == "EXP":
        x = np.clip(x, -80, 80)
    if op in ("SIN", "COS", "TAN"):
        x = x[:, np.abs(x[0]) < 10]
    x = x.astype(np.float32).astype(np.float64)
    n, k = x.shape[1], x.shape[0]
    y32, J = o.jacobian([x], scalar=32)
    assert np.array_equal(y32[0], o.evaluate([x], 32)[0], equal_nan=True)
    assert np.array_equal(J.astype(np.float32).astype(np.float64), J, equal_nan=True)
    for i in range(n):
        with mpmath.workdps(40):
            a = mpmath.mpf(float(x[0, i]))
            b = mpmath.mpf(float(x[1, i])) if k > 1 else None
            da, db = DERIV[op](a, b)
            refs = [da] + ([db] if k > 1 else [])
        for j, r in enumerate(refs):
            r = float(r)
            got = J[0, j, i]
            if not np.isfinite(r) or abs(r) > 1e30:
                continue
            # TAN/TANH form 1 +- v^2 from the rounded value v; POW's
            # derivatives carry the rounding of log(a) and pow() scaled by |b log a|
            rel = 8 * 2.0 ** -24
            if op == "TAN":
                rel *= 1 + abs(float(x[0, i])) / (1e-3 + abs(math.cos(float(x[0, i]))))
            if op == "POW":
                rel *= 4 + abs(float(x[1, i]) * math.log(abs(float(x[0, i])) + 1e-300))
            atol = 4 * 2.0 ** -23 if op == "TANH" else 1e-37
            assert abs(got - r) <= rel * abs(r) + atol, (op, j, float(x[0, i]), got, r)


def test_binary32_dual_pendulum_close_to_binary64(tmp_path):
    """On the pendulum step the binary32 Jacobian differs from the binary64
    one (binary32 arithmetic was used) by a small relative amount."""
    from workloads import inputs
    from workloads.pendulum import pendulum
    path = tmp_path / "p.xgp"
    pendulum(7).save(path)
    o = OProg(path)
    x = inputs.pendulum_state(5, 7, 16).astype(np.float32).astype(np.float64)
    _, J64 = o.jacobian([x], threads=4)
    _, J32 = o.jacobian([x], threads=4, scalar=32)
    scale = np.abs(J64).max()
    d = np.abs(J32 - J64).max() / scale
    assert 0 < d < 1e-4, d


def _bad(tmp_path, instrs, nnz_out=(1,), n_work=2):
    p = Program("bad", "f64", n_work, [1], list(nnz_out), [1.5], instrs)
    path = tmp_path / "bad.xgp"
    p.save(path)
    with pytest.raises(OracleError) as e:
        OProg(path)
    return str(e.value)


def test_validation_errors(tmp_path):
    assert "read before write" in _bad(tmp_path, [("ADD", 0, 1, 1), ("OUTPUT", 0, 0, 0)])
    assert "never written" in _bad(tmp_path, [("INPUT", 0, 0, 0), ("OUTPUT", 0, 0, 0)], nnz_out=(2,))
    assert "input index" in _bad(tmp_path, [("INPUT", 0, 0, 3), ("OUTPUT", 0, 0, 0)])
    assert "slot out of range" in _bad(tmp_path, [("INPUT", 5, 0, 0), ("OUTPUT", 0, 5, 0)])
    assert "const index" in _bad(tmp_path, [("CONST", 0, 4, -1), ("OUTPUT", 0, 0, 0)])
    path = tmp_path / "u.xgp"
    path.write_text("xgprog 1\nname u\ndtype f64\nn_work 1\ninputs 1 1\noutputs 1 1\nconsts 0\n"
                    "instrs 2\nINPUT 0 0 0\nFOO 0 0 0\nend\n")
    with pytest.raises(OracleError, match="unknown op"):
        OProg(path)


def test_last_output_write_wins(tmp_path):
    ins = [("INPUT", 0, 0, 0), ("OUTPUT", 0, 0, 0), ("NEG", 1, 0, -1), ("OUTPUT", 0, 1, 0)]
    p = tmp_path / "o.xgp"
    Program("o", "f64", 2, [1], [1], [], ins).save(p)
    y = OProg(p).evaluate([np.array([[1.0, -2.0]])])[0]
    assert np.array_equal(y, [[-1.0, 2.0]])


def test_threads_do_not_change_results(tmp_path):
    from workloads.rdag import rdag
    from workloads import inputs
    p = tmp_path / "r.xgp"
    rdag(5, 8, 300).save(p)
    o = OProg(p)
    x = inputs.uniform(9, 8, 1001)
    assert np.array_equal(o.evaluate([x], 64, threads=1)[0], o.evaluate([x], 64, threads=7)[0])


@pytest.mark.parametrize("op", UNARY + BINARY)
def test_f32_tagged_instruction(op, tmp_path):
    """Inside an f64 program an f32-tagged instruction rounds its operands to
    binary32, computes in binary32 and widens the result: exactly the float
    evaluation of the same operation (mpmath-pinned above)."""
    base = one_op_program(op)
    tagged = Program(base.name, "f64", base.n_work, base.nnz_in, base.nnz_out, [], base.instrs,
                     prec={len(base.instrs) - 2: "f32"})
    p = tmp_path / "t.xgp"
    tagged.save(p)
    rng = np.random.default_rng(5)
    x = grid(op, rng, 200)
    if op == "EXP":
        x = np.clip(x, -80, 80)
    x32 = x.astype(np.float32).astype(np.float64)
    ok = np.all(np.isfinite(x32), axis=0)
    x, x32 = x[:, ok], x32[:, ok]
    y = OProg(p).evaluate([x], 64)[0][0]          # operands rounded inside
    q = tmp_path / "u.xgp"
    base.save(q)
    r = OProg(q).evaluate([x32], 32)[0][0]        # float evaluation
    assert np.array_equal(y, r, equal_nan=True), op


def test_f32_tag_rejected_outside_f64(tmp_path):
    p = Program("t", "f32", 2, [1], [1], [], [("INPUT", 0, 0, 0), ("SIN", 1, 0, -1),
                                              ("OUTPUT", 0, 1, 0)], prec={1: "f32"})
    path = tmp_path / "t.xgp"
    p.save(path)
    with pytest.raises(OracleError, match="f32 tag"):
        OProg(path)
