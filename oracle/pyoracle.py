"""ctypes wrapper of the oracle interpreter (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads ``oracle/liboracle.so`` (built by
``oracle/Makefile``) and exposes:

* :func:`evaluate` -- outputs of a program file for N instances in float
  (32), double (64) or x87 long double (80) arithmetic;
* :func:`jvp` / :func:`jacobian` / :func:`vjp` -- forward-mode dual-number
  derivatives (exact up to rounding).

Arrays are structure-of-arrays: one float64 array of shape (nnz, N) per
argument.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_P = ctypes.c_void_p
_LL = ctypes.c_longlong


def build() -> str:
    subprocess.run(["make", "-s", "-C", _HERE], check=True)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(
                os.path.join(_HERE, "xg_oracle.cpp")):
            build()
        L = ctypes.CDLL(_LIB)
        L.xo_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(_P)]
        L.xo_load.restype = ctypes.c_int
        L.xo_free.argtypes = [_P]
        L.xo_last_error.restype = ctypes.c_char_p
        L.xo_info.argtypes = [_P] + [ctypes.POINTER(_LL)] * 6
        L.xo_eval.argtypes = [_P, ctypes.c_int, _LL, ctypes.POINTER(_P), ctypes.POINTER(_LL),
                              ctypes.POINTER(_P), ctypes.POINTER(_LL), ctypes.c_int]
        L.xo_jvp.argtypes = [_P, ctypes.c_int, _LL, ctypes.POINTER(_P), ctypes.POINTER(_LL),
                             ctypes.POINTER(_P), ctypes.POINTER(_LL), ctypes.c_int, _P, _P,
                             ctypes.c_int]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


class Program:
    """A program file loaded and validated by the oracle's own parser."""

    def __init__(self, path):
        L = lib()
        h = _P()
        if L.xo_load(str(path).encode(), ctypes.byref(h)) != 0:
            raise OracleError(L.xo_last_error().decode())
        self._h = h
        n_in, n_out, nw, ni = _LL(), _LL(), _LL(), _LL()
        L.xo_info(h, ctypes.byref(n_in), ctypes.byref(n_out), None, None, ctypes.byref(nw),
                  ctypes.byref(ni))
        a = (_LL * max(n_in.value, 1))()
        b = (_LL * max(n_out.value, 1))()
        L.xo_info(h, ctypes.byref(n_in), ctypes.byref(n_out), a, b, None, None)
        self.nnz_in = [a[i] for i in range(n_in.value)]
        self.nnz_out = [b[i] for i in range(n_out.value)]
        self.n_work = nw.value
        self.n_instr = ni.value

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.xo_free(self._h)
            self._h = None

    def _ptrs(self, xs, nnz, n, writable):
        if len(xs) != len(nnz):
            raise ValueError("wrong number of arguments")
        arrs = []
        for x, k in zip(xs, nnz):
            x = np.asarray(x, dtype=np.float64)
            if x.shape != (k, n):
                raise ValueError(f"argument shape {x.shape} != {(k, n)}")
            if writable:
                if not x.flags.c_contiguous:
                    raise ValueError("output must be C-contiguous")
            else:
                x = np.ascontiguousarray(x)
            arrs.append(x)
        ptrs = (_P * max(len(arrs), 1))(*[a.ctypes.data for a in arrs])
        lds = (_LL * max(len(arrs), 1))(*[n for _ in arrs])
        return arrs, ptrs, lds

    def evaluate(self, xs, scalar: int = 64, threads: int = 1):
        n = np.asarray(xs[0]).shape[1] if xs else 0
        ins, pin, ldi = self._ptrs(xs, self.nnz_in, n, False)
        outs = [np.full((k, n), np.nan) for k in self.nnz_out]
        _, pout, ldo = self._ptrs(outs, self.nnz_out, n, True)
        if lib().xo_eval(self._h, scalar, n, pin, ldi, pout, ldo, threads) != 0:
            raise OracleError(lib().xo_last_error().decode())
        return outs

    def jvp(self, xs, tangents, threads: int = 1, scalar: int = 64):
        """tangents: array (K, tot_in, N).  Returns (outputs, (K, tot_out, N)).
        scalar 32 carries values and tangents in binary32."""
        n = np.asarray(xs[0]).shape[1]
        tin = np.ascontiguousarray(tangents, dtype=np.float64)
        K = tin.shape[0]
        if tin.shape != (K, sum(self.nnz_in), n):
            raise ValueError("tangent shape")
        ins, pin, ldi = self._ptrs(xs, self.nnz_in, n, False)
        outs = [np.full((k, n), np.nan) for k in self.nnz_out]
        _, pout, ldo = self._ptrs(outs, self.nnz_out, n, True)
        tout = np.full((K, sum(self.nnz_out), n), np.nan)
        if lib().xo_jvp(self._h, scalar, n, pin, ldi, pout, ldo, K, tin.ctypes.data,
                        tout.ctypes.data, threads) != 0:
            raise OracleError(lib().xo_last_error().decode())
        return outs, tout

    def jacobian(self, xs, threads: int = 1, scalar: int = 64):
        """Full Jacobian (tot_out, tot_in, N) by dual numbers."""
        n = np.asarray(xs[0]).shape[1]
        m = sum(self.nnz_in)
        seeds = np.zeros((m, m, n))
        for e in range(m):
            seeds[e, e, :] = 1.0
        outs, t = self.jvp(xs, seeds, threads, scalar)
        return outs, np.ascontiguousarray(np.transpose(t, (1, 0, 2)))

    def vjp(self, xs, ybar, threads: int = 1, scalar: int = 64):
        """x_bar = J^T y_bar per instance (ybar: list of (nnz_out, N)); the
        Jacobian in the given scalar type, the product with y_bar in double."""
        outs, J = self.jacobian(xs, threads, scalar)
        yb = np.concatenate([np.asarray(y, dtype=np.float64) for y in ybar], axis=0)
        xb = np.einsum("oin,on->in", J, yb)
        res, off = [], 0
        for k in self.nnz_in:
            res.append(xb[off:off + k])
            off += k
        return outs, res


def evaluate_program(prog, xs, scalar=64, threads=1, tmpdir=None):
    """Save a workloads.Program to a temporary file and evaluate it."""
    import tempfile
    d = tmpdir or tempfile.mkdtemp(prefix="xgo_")
    path = os.path.join(d, f"{prog.name}.xgp")
    prog.save(path)
    return Program(path).evaluate(xs, scalar=scalar, threads=threads)
