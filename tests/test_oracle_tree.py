"""Pin of the oracle's sequential slot semantics against a demand-driven
recursive evaluator on tiny random programs.

The recursive evaluator never walks the instruction list forwards: the
value of slot s just before instruction t is the result of the last
instruction before t that wrote s, evaluated recursively from its own
operands (tree evaluation).  Programs use very few slots, so operands and
results are reused and overwritten in place, and OUTPUT instructions
appear anywhere (the last write of an output element wins).

Arithmetic uses numpy float64 (IEEE, correctly rounded, no contraction)
and the same C library's transcendental routines through ctypes, so the
two evaluators must agree bitwise.
"""

import ctypes
import ctypes.util

import numpy as np
from hypothesis import given, settings, strategies as st

from oracle.pyoracle import Program as OProg
from workloads.tracer import Program

_m = ctypes.CDLL(ctypes.util.find_library("m"))
for _f in ("sin", "cos", "tanh", "atan", "exp", "fmin", "fmax", "sqrt"):
    getattr(_m, _f).restype = ctypes.c_double
    getattr(_m, _f).argtypes = [ctypes.c_double] * (2 if _f in ("fmin", "fmax") else 1)

U = ["NEG", "SQ", "SIN", "COS", "TANH", "ATAN", "FABS", "SQRT", "EXP"]
B = ["ADD", "SUB", "MUL", "DIV", "FMIN", "FMAX", "LT", "LE"]


def ref_op(op, a, b):
    f = np.float64
    with np.errstate(all="ignore"):
        if op == "ADD":
            return f(a) + f(b)
        if op == "SUB":
            return f(a) - f(b)
        if op == "MUL":
            return f(a) * f(b)
        if op == "DIV":
            return f(a) / f(b)
        if op == "NEG":
            return -f(a)
        if op == "SQ":
            return f(a) * f(a)
        if op == "FABS":
            return np.abs(f(a))
        if op == "LT":
            return f(1.0) if a < b else f(0.0)
        if op == "LE":
            return f(1.0) if a <= b else f(0.0)
        if op in ("FMIN", "FMAX"):
            return f(getattr(_m, op.lower())(float(a), float(b)))
        return f(getattr(_m, op.lower())(float(a)))


@st.composite
def programs(draw):
    n_in = draw(st.integers(1, 3))
    W = draw(st.integers(2, 4))
    n_out = draw(st.integers(1, 3))
    consts = [draw(st.floats(-3, 3, allow_nan=False)) for _ in range(2)]
    ins = []
    written = set()
    for s in range(W):  # start by defining every slot
        if draw(st.booleans()) or s == 0:
            ins.append(("INPUT", s, 0, draw(st.integers(0, n_in - 1))))
        else:
            ins.append(("CONST", s, draw(st.integers(0, 1)), -1))
        written.add(s)
    outs_written = set()
    for _ in range(draw(st.integers(1, 14))):
        kind = draw(st.integers(0, 9))
        if kind == 0:
            e = draw(st.integers(0, n_out - 1))
            ins.append(("OUTPUT", 0, draw(st.integers(0, W - 1)), e))
            outs_written.add(e)
            continue
        out = draw(st.integers(0, W - 1))
        a = draw(st.integers(0, W - 1))
        if kind <= 4:
            ins.append((draw(st.sampled_from(U)), out, a, -1))
        else:
            ins.append((draw(st.sampled_from(B)), out, a, draw(st.integers(0, W - 1))))
    for e in range(n_out):
        if e not in outs_written or draw(st.booleans()):
            ins.append(("OUTPUT", 0, draw(st.integers(0, W - 1)), e))
    return Program("tree", "f64", W, [n_in], [n_out], consts, ins)


def tree_eval(p: Program, x):
    """Evaluate outputs by recursion from the last writes, never forwards."""
    memo = {}

    def slot_value(s, t):  # value of slot s just before instruction t
        for u in range(t - 1, -1, -1):
            op, out, a, b = p.instrs[u]
            if op != "OUTPUT" and out == s:
                return instr_value(u)
        raise AssertionError("read before write")

    def instr_value(u):
        if u in memo:
            return memo[u]
        op, out, a, b = p.instrs[u]
        if op == "INPUT":
            v = np.float64(x[b])
        elif op == "CONST":
            v = np.float64(p.consts[a])
        else:
            va = slot_value(a, u)
            vb = slot_value(b, u) if b >= 0 and op in B else None
            v = ref_op(op, va, vb)
        memo[u] = v
        return v

    res = []
    for e in range(p.nnz_out[0]):
        last = max(u for u, ins in enumerate(p.instrs) if ins[0] == "OUTPUT" and ins[3] == e)
        res.append(slot_value(p.instrs[last][2], last))
    return np.array(res, dtype=np.float64)


def same(a, b):
    return (a == b) or (np.isnan(a) and np.isnan(b))


@settings(max_examples=600, deadline=None)
@given(programs(), st.integers(0, 2**31))
def test_sequential_semantics_match_tree_evaluation(tmp_path_factory, prog, seed):
    d = tmp_path_factory.mktemp("t")
    path = d / "t.xgp"
    prog.save(path)
    o = OProg(path)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-2, 2, size=(prog.nnz_in[0], 3))
    y = o.evaluate([x], 64)[0]
    for i in range(3):
        r = tree_eval(prog, x[:, i])
        for e in range(len(r)):
            assert same(y[e, i], r[e]), (prog.instrs, x[:, i], e, y[e, i], r[e])
