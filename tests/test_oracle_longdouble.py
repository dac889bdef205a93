"""Pins of the oracle's x87 long double mode (scalar 80) against mpmath.

The inherent-sensitivity gates compare the oracle in long double with the
oracle in double; they mean something only if the long double mode really
carries a 64-bit significand through every operation.  Its outputs are
rounded to double, so a plain comparison of outputs cannot tell the two
modes apart.  Each check here therefore evaluates a residual program

    r = op(x[, y]) - c,   c = the double nearest to the exact op(x[, y])

(c is a second input).  In long double, op(x) is rounded to 64 significant
bits and the subtraction is exact (both operands lie within one double ulp of
each other), so r holds the bits of op(x) below double precision, and r
itself fits in a double exactly.  The reference is the same residual of
mpmath's value rounded to a 64-bit significand.  Gates: the correctly
rounded operations (+, -, *, /, sqrt, sq) bitwise; the library functions
within 2 units of the 64-bit significand (2^-62 relative).  A double
evaluation of the same residual is 0 or one double ulp away, i.e. off by up
to 2^10 units of the 64-bit significand, and must fail the same gate.
"""

import mpmath
import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from workloads.tracer import Program

from .test_oracle_ops import BINARY, UNARY, grid, mp_ref

EXACT80 = {"ADD", "SUB", "MUL", "DIV", "SQRT", "SQ"}
# operations whose result is one of the operands (or 0/1): no residual below
# double precision exists, so they carry no information here
TRIVIAL = {"NEG", "FABS", "FMIN", "FMAX", "LT", "LE"}
OPS = [op for op in UNARY + BINARY if op not in TRIVIAL]


def residual_program(op):
    if op in UNARY:
        ins = [("INPUT", 0, 0, 0), ("INPUT", 1, 1, 0), (op, 2, 0, -1), ("SUB", 2, 2, 1),
               ("OUTPUT", 0, 2, 0)]
        return Program(f"res_{op}", "f64", 3, [1, 1], [1], [], ins)
    ins = [("INPUT", 0, 0, 0), ("INPUT", 1, 0, 1), ("INPUT", 2, 1, 0), (op, 0, 0, 1),
           ("SUB", 0, 0, 2), ("OUTPUT", 0, 0, 0)]
    return Program(f"res_{op}", "f64", 3, [2, 1], [1], [], ins)


def references(op, x):
    """(c, r_ref, scale): the double nearest to the exact value, the exact
    value rounded to a 64-bit significand minus c, and |exact value|."""
    n = x.shape[1]
    c = np.empty(n)
    r = np.empty(n)
    mag = np.empty(n)
    for i in range(n):
        with mpmath.workdps(60):
            a = mpmath.mpf(float(x[0, i]))
            b = mpmath.mpf(float(x[1, i])) if x.shape[0] > 1 else None
            v = mp_ref(op, a, b)
            with mpmath.workprec(53):
                vc = +v
            with mpmath.workprec(64):
                v64 = +v
            c[i] = float(vc)
            r[i] = float(v64 - vc)  # exact: few significant bits
            mag[i] = float(abs(v))
    return c, r, mag


def _points(op):
    rng = np.random.default_rng(11)
    x = grid(op, rng, n=300)
    if op == "EXP":
        x = np.clip(x, -700, 700)
    if op == "TAN":  # keep away from the poles, where 2 units of long double are not 2 units of the result
        x = x[:, np.abs(np.cos(x[0])) > 1e-3]
    return x


def _units(op, scalar, tmp_path):
    """Error of the residual in units of 2^-63 |op(x)| (the 64-bit
    significand's half-binade unit), per point."""
    x = _points(op)
    c, r_ref, mag = references(op, x)
    ok = np.isfinite(c) & (mag > 1e-300) & (mag < 1e300)
    x, c, r_ref, mag = x[:, ok], c[ok], r_ref[ok], mag[ok]
    path = tmp_path / f"r_{op}.xgp"
    residual_program(op).save(path)
    o = OProg(path)
    xs = [x, c[None, :]]
    r = o.evaluate(xs, scalar)[0][0]
    unit = np.ldexp(1.0, -63) * mag
    return np.abs(r - r_ref) / unit, r, r_ref


@pytest.mark.parametrize("op", OPS)
def test_long_double_carries_64_bit_significand(op, tmp_path):
    err80, r, r_ref = _units(op, 80, tmp_path)
    if op in EXACT80:
        assert np.array_equal(r, r_ref), (op, np.flatnonzero(r != r_ref)[:5])
    else:
        assert err80.max() <= 2.0, (op, err80.max())
    # the same gate rejects a double-precision evaluation of the residual
    err64, _, _ = _units(op, 64, tmp_path)
    assert np.mean(err64 > 2.0) > 0.5, (op, np.mean(err64 > 2.0))


def test_long_double_cancellation(tmp_path):
    """(x + y) - x recovers y = 2^-60 x in long double (64-bit significand)
    and loses it in double."""
    ins = [("INPUT", 0, 0, 0), ("INPUT", 1, 0, 1), ("ADD", 2, 0, 1), ("SUB", 2, 2, 0),
           ("OUTPUT", 0, 2, 0)]
    path = tmp_path / "cancel.xgp"
    Program("cancel", "f64", 3, [2], [1], [], ins).save(path)
    x = np.array([1.0, 3.0, -7.5, 1024.0])  # short significands: x + y is exact in 64 bits
    y = np.ldexp(x, -60)
    o = OProg(path)
    assert np.array_equal(o.evaluate([np.stack([x, y])], 80)[0][0], y)
    assert np.array_equal(o.evaluate([np.stack([x, y])], 64)[0][0], np.zeros(4))
