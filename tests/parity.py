"""The parity rule shared by the GPU tests.

For output component j and instance n with reference r:
    err[j, n] = |y[j, n] - r[j, n]| / max(|r[j, n]|, s_j),
    s_j = RMS over instances of r[j, :]   (s_j = 1 if it is 0).
The gate is on max err.  Tolerances: fp64 1e-12 (fp64 MPC 1e-9); fp32
max(1e-5, 4 e32) with e32 the same measure between the oracle's float and
double evaluations of the same (float-rounded) inputs; for fp32 gradients
e32 compares the oracle's binary32 and binary64 dual-number gradients.
"""

import numpy as np

TOL_F64 = 1e-12
TOL_F64_MPC = 1e-9
TOL_F32 = 1e-5


def err(y, r):
    y = np.asarray(y, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    s = np.sqrt(np.mean(r * r, axis=1, keepdims=True))
    s[s == 0] = 1.0
    return np.abs(y - r) / np.maximum(np.abs(r), s)


def max_err(ys, rs):
    return max(float(err(y, r).max()) if y.size else 0.0 for y, r in zip(ys, rs))


def report(ys, rs, tol):
    e = np.concatenate([err(y, r).ravel() for y, r in zip(ys, rs)])
    return {"max": float(e.max()) if e.size else 0.0,
            "p99": float(np.quantile(e, 0.99)) if e.size else 0.0,
            "over": int((e > tol).sum())}


def f32_tol(o, xs):
    """max(1e-5, 4 e32) for a binary32 forward evaluation at inputs xs."""
    return max(TOL_F32, 4 * max_err(o.evaluate(xs, 32, threads=8), o.evaluate(xs, 64, threads=8)))


def f32_grad_tol(o, xs, ybars):
    """max(1e-5, 4 e32) for a binary32 gradient J^T y_bar at inputs xs."""
    _, g64 = o.vjp(xs, ybars, threads=8)
    _, g32 = o.vjp(xs, ybars, threads=8, scalar=32)
    return max(TOL_F32, 4 * max_err(g32, g64))
