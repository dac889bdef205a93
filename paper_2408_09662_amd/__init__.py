"""xg: batched evaluation of straight-line scalar programs on one MI355X.

Thin Python binding of the C-ABI library ``libxg.so`` (declared in
``include/xg.h``).  Every evaluation runs in the library's generated HIP
kernels; this module only marshals arguments.  PyTorch provides device
memory and streams.  If the native library is missing the import fails: there
is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _abi
from ._abi import XgError, lib, OPS, OP_ID, XG_F32, XG_F64  # noqa: F401

__all__ = ["Program", "Batch", "Graph", "XgFunction", "autotune", "autotune_adjoint", "autotune_batch", "autotune_batch_precompile", "autotune_precompile", "capture_eval", "capture_rollout", "load_program_file", "lib", "XgError"]


def load_program_file(path):
    """Parse a program file into plain arrays (the binding's own parser).

    Returns dict(name, dtype, n_work, nnz_in, nnz_out, consts, instr) where
    instr is an int32 array (n_instr, 4) of (op id, out, a, b)."""
    with open(path) as f:
        toks = f.read().split("\n")
    it = iter(toks)

    def nxt():
        while True:
            line = next(it).strip()
            if line:
                return line

    head = nxt().split()
    if head != ["xgprog", "1"]:
        raise XgError(f"{path}: not an xg program file")
    d = {}
    for key in ("name", "dtype", "n_work"):
        k, v = nxt().split(maxsplit=1)
        if k != key:
            raise XgError(f"{path}: expected {key}")
        d[key] = v
    d["n_work"] = int(d["n_work"])
    for key in ("inputs", "outputs"):
        parts = nxt().split()
        if parts[0] != key:
            raise XgError(f"{path}: expected {key}")
        k = int(parts[1])
        d["nnz_in" if key == "inputs" else "nnz_out"] = [int(v) for v in parts[2:2 + k]]
    parts = nxt().split()
    nc = int(parts[1])
    d["consts"] = np.array([float.fromhex(nxt()) for _ in range(nc)], dtype=np.float64)
    parts = nxt().split()
    ni = int(parts[1])
    instr = np.empty((ni, 4), dtype=np.int32)
    for i in range(ni):
        o, a, b, c = nxt().split()
        if o not in OP_ID:
            raise XgError(f"{path}: unknown op {o} at instruction {i}")
        instr[i] = (OP_ID[o], int(a), int(b), int(c))
    tok = nxt()
    prec = None
    if tok.startswith("prec"):
        npr = int(tok.split()[1])
        prec = np.zeros(ni, dtype=np.int8)
        for _ in range(npr):
            i, v = nxt().split()
            if v != "f32":
                raise XgError(f"{path}: bad precision tag {v}")
            prec[int(i)] = 32
        tok = nxt()
    if tok != "end":
        raise XgError(f"{path}: missing end")
    d["instr"] = instr
    d["prec"] = prec
    return d


def _from_workload(prog):
    instr = np.array([(OP_ID[o], p, a, b) for (o, p, a, b) in prog.instrs], dtype=np.int32)
    prec = None
    if getattr(prog, "prec", None):
        prec = np.zeros(len(prog.instrs), dtype=np.int8)
        for i, v in prog.prec.items():
            prec[i] = 32 if v == "f32" else 64
    return dict(name=prog.name, dtype=prog.dtype, n_work=prog.n_work, nnz_in=list(prog.nnz_in),
                nnz_out=list(prog.nnz_out), consts=np.array(prog.consts, dtype=np.float64),
                instr=instr.reshape(-1, 4), prec=prec)


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptrs(tensors, n, dtype, nnz, what="argument"):
    """ctypes arrays of device pointers and pitches for one argument list.

    Checked before any launch: one tensor per argument (len(nnz) of them),
    each a CUDA tensor of the program's dtype with shape (nnz[i], >= n) and
    unit stride over instances.  The library reads or writes nnz[i] rows at
    the returned pitch, so a short list or a tensor with too few rows is an
    error here, never an out-of-bounds access there."""
    torch = _torch()
    tensors = list(tensors)
    k = len(nnz)
    if len(tensors) != k:
        raise XgError(f"expected {k} {what} tensors, got {len(tensors)}")
    P = (ctypes.c_void_p * max(k, 1))()
    L = (ctypes.c_int64 * max(k, 1))()
    for i, t in enumerate(tensors):
        if t is None:
            if nnz[i] != 0:
                raise XgError(f"{what} {i} is None but has {nnz[i]} elements")
            P[i] = None
            L[i] = n
            continue
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise XgError(f"{what} {i} must be a CUDA (HIP) tensor")
        if t.dtype != dtype:
            raise XgError(f"{what} {i}: dtype {t.dtype} does not match the program's {dtype}")
        if t.dim() != 2 or t.stride(1) != 1 or t.shape[1] < n:
            raise XgError(f"{what} {i} must be 2-D (nnz, N >= {n}) with unit stride over instances")
        if t.shape[0] != nnz[i]:
            raise XgError(f"{what} {i} has {t.shape[0]} rows; the program's argument has {nnz[i]}")
        P[i] = t.data_ptr()
        L[i] = t.stride(0) if t.shape[0] > 1 else max(n, t.shape[1])
    return P, L


class Program:
    """A loaded program.  `src` is a program file path, a workloads.Program,
    or the dict returned by :func:`load_program_file`.

    options: dict of xg_options fields (block, ipt, chunk_ops, reg_budget,
    lds_slots, strict, eager, adj_seg_ops, verbose)."""

    def __init__(self, src, **options):
        if isinstance(src, (str, os.PathLike)):
            d = load_program_file(src)
        elif isinstance(src, dict):
            d = src
        else:
            d = _from_workload(src)
        self.name = d["name"]
        self.dtype = d["dtype"]
        self.nnz_in = list(d["nnz_in"])
        self.nnz_out = list(d["nnz_out"])
        self.options = dict(options)
        L = lib()
        nin = (ctypes.c_int32 * max(len(self.nnz_in), 1))(*self.nnz_in)
        nout = (ctypes.c_int32 * max(len(self.nnz_out), 1))(*self.nnz_out)
        instr = np.ascontiguousarray(d["instr"], dtype=np.int32)
        consts = np.ascontiguousarray(d["consts"], dtype=np.float64)
        prec = d.get("prec")
        if prec is not None:
            prec = np.ascontiguousarray(prec, dtype=np.int8)
            if prec.shape != (instr.shape[0],):
                raise XgError("prec must have one entry per instruction")
        desc = _abi.ProgramDesc(
            n_in=len(self.nnz_in), nnz_in=nin, n_out=len(self.nnz_out), nnz_out=nout,
            n_work=int(d["n_work"]), n_instr=instr.shape[0],
            instr=instr.ctypes.data_as(ctypes.c_void_p), n_const=consts.shape[0],
            consts=consts.ctypes.data_as(ctypes.c_void_p),
            dtype=XG_F64 if self.dtype == "f64" else XG_F32,
            prec=prec.ctypes.data_as(ctypes.c_void_p) if prec is not None else None)
        self._prec_keep = prec
        opts = _abi.make_options(options)
        h = ctypes.c_void_p()
        _abi.check(L.xg_program_load(ctypes.byref(desc), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _abi is not None and _abi._lib is not None:
            # (at interpreter exit the module globals may already be gone)
            _abi._lib.xg_program_free(h)
            self._h = None

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float64 if self.dtype == "f64" else torch.float32

    def info(self, mode: int = 0) -> dict:
        inf = _abi.Info()
        _abi.check(lib().xg_program_info(self._h, mode, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _abi.Info._fields_}

    def effective_options(self, mode: int = 0) -> dict:
        """The options `mode` runs with (defaults resolved; autotuned if
        tuned: autotune() sets mode 0, autotune_adjoint() modes 1 and 2)."""
        o = _abi.Options()
        _abi.check(lib().xg_program_options(self._h, mode, ctypes.byref(o)))
        return {f: getattr(o, f) for f in _abi.OPTION_FIELDS}

    def workspace_bytes(self, n: int, mode: int = 0) -> int:
        b = ctypes.c_size_t()
        _abi.check(lib().xg_workspace_bytes(self._h, n, mode, ctypes.byref(b)))
        return b.value

    def precompile(self, mode: int = 0) -> None:
        _abi.check(lib().xg_precompile(self._h, mode))

    def compile(self, mode: int = 0) -> None:
        _abi.check(lib().xg_compile(self._h, mode))

    def workspace(self, n: int, mode: int = 0):
        """A cached device workspace (torch uint8 tensor) or None."""
        nb = self.workspace_bytes(n, mode)
        if nb == 0:
            return None
        key = (mode, _torch().cuda.current_device())
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nb:
            ws = _torch().empty(nb, dtype=_torch().uint8, device="cuda")
            self._ws[key] = ws
        return ws

    def alloc_outputs(self, n: int):
        torch = _torch()
        return [torch.empty((k, n), dtype=self.torch_dtype, device="cuda") for k in self.nnz_out]

    def _n_of(self, tensors, n):
        if n is not None:
            return int(n)
        for t in tensors or ():
            if t is not None and hasattr(t, "shape") and len(t.shape) == 2:
                return int(t.shape[1])
        raise XgError("cannot tell the instance count: pass n")

    def eval(self, inputs, outputs=None, n=None, stream=None, workspace=None):
        """y = P(x) for all instances.  inputs: list of (nnz, N) CUDA tensors."""
        if len(inputs) != len(self.nnz_in):
            raise XgError(f"expected {len(self.nnz_in)} input tensors, got {len(inputs)}")
        n = self._n_of(list(inputs) + list(outputs or []), n)
        if outputs is None:
            outputs = self.alloc_outputs(n)
        pi, li = _ptrs(inputs, n, self.torch_dtype, self.nnz_in, "input")
        po, lo = _ptrs(outputs, n, self.torch_dtype, self.nnz_out, "output")
        ws = workspace if workspace is not None else self.workspace(n, 0)
        _abi.check(lib().xg_eval(self._h, n, pi, li, po, lo,
                                 ctypes.c_void_p(ws.data_ptr() if ws is not None else 0),
                                 _stream_handle(stream)))
        return outputs

    def bind_eval(self, inputs, outputs, n=None, stream=None, workspace=None):
        """A zero-argument callable that launches y = P(x) on fixed buffers
        (arguments are marshalled once; each call is one C-ABI call)."""
        n = self._n_of(inputs, n)
        pi, li = _ptrs(inputs, n, self.torch_dtype, self.nnz_in, "input")
        po, lo = _ptrs(outputs, n, self.torch_dtype, self.nnz_out, "output")
        ws = workspace if workspace is not None else self.workspace(n, 0)
        wsp = ctypes.c_void_p(ws.data_ptr() if ws is not None else 0)
        st = _stream_handle(stream)
        f = lib().xg_eval
        h = self._h
        keep = (inputs, outputs, ws)

        def run():
            _abi.check(f(h, n, pi, li, po, lo, wsp, st))
            return keep
        return run

    def eval_adjoint(self, inputs, seeds, grads=None, outputs=None, with_outputs=False, n=None,
                     stream=None, workspace=None):
        """x_bar = J^T y_bar (and y if with_outputs).  Returns grads or (grads, outputs)."""
        torch = _torch()
        for lst, k, what in ((inputs, self.nnz_in, "input"), (seeds, self.nnz_out, "seed")):
            if len(lst) != len(k):
                raise XgError(f"expected {len(k)} {what} tensors, got {len(lst)}")
        n = self._n_of(inputs, n)
        if grads is None:
            grads = [torch.empty((k, n), dtype=self.torch_dtype, device="cuda") for k in self.nnz_in]
        if with_outputs and outputs is None:
            outputs = self.alloc_outputs(n)
        mode = 2 if with_outputs else 1
        pi, li = _ptrs(inputs, n, self.torch_dtype, self.nnz_in, "input")
        ps, ls = _ptrs(seeds, n, self.torch_dtype, self.nnz_out, "seed")
        pg, lg = _ptrs(grads, n, self.torch_dtype, self.nnz_in, "gradient")
        if with_outputs:
            po, lo = _ptrs(outputs, n, self.torch_dtype, self.nnz_out, "output")
        else:
            po, lo = None, None
        ws = workspace if workspace is not None else self.workspace(n, mode)
        _abi.check(lib().xg_eval_adjoint(self._h, n, pi, li, ps, ls, po, lo, pg, lg,
                                         ctypes.c_void_p(ws.data_ptr() if ws is not None else 0),
                                         _stream_handle(stream)))
        return (grads, outputs) if with_outputs else grads

    def eval_adjoint_noalloc(self, inputs, seeds, grads, outputs=None, n=None, stream=None):
        """eval_adjoint on caller-provided buffers with the library's fixed
        device scratch array as the workspace (xg_eval_adjoint_noalloc):
        nothing is allocated, so the mode's kernels must already be loaded
        (Program.compile(1), or compile(2) when `outputs` is given)."""
        for lst, k, what in ((inputs, self.nnz_in, "input"), (seeds, self.nnz_out, "seed"),
                             (grads, self.nnz_in, "gradient")):
            if len(lst) != len(k):
                raise XgError(f"expected {len(k)} {what} tensors, got {len(lst)}")
        n = self._n_of(inputs, n)
        pi, li = _ptrs(inputs, n, self.torch_dtype, self.nnz_in, "input")
        ps, ls = _ptrs(seeds, n, self.torch_dtype, self.nnz_out, "seed")
        pg, lg = _ptrs(grads, n, self.torch_dtype, self.nnz_in, "gradient")
        if outputs is not None:
            po, lo = _ptrs(outputs, n, self.torch_dtype, self.nnz_out, "output")
        else:
            po, lo = None, None
        _abi.check(lib().xg_eval_adjoint_noalloc(self._h, n, pi, li, ps, ls, po, lo, pg, lg,
                                                 _stream_handle(stream)))
        return (grads, outputs) if outputs is not None else grads


def _make_function():
    torch = _torch()

    class XgFunction(torch.autograd.Function):
        """y = P(x) with reverse-mode gradients from the library's adjoint
        kernels.  Single input and single output argument programs: x is
        (nnz_in, N), y is (nnz_out, N).  Only x is saved for backward; the
        adjoint recomputes the forward values it needs."""

        @staticmethod
        def forward(ctx, prog, x):
            ctx.prog = prog
            ctx.save_for_backward(x)
            return prog.eval([x.contiguous()])[0]

        @staticmethod
        def backward(ctx, gy):
            (x,) = ctx.saved_tensors
            g = ctx.prog.eval_adjoint([x.contiguous()], [gy.contiguous()])[0]
            return None, g

    return XgFunction


class _LazyFunction:
    _f = None

    def __getattr__(self, k):
        if _LazyFunction._f is None:
            _LazyFunction._f = _make_function()
        return getattr(_LazyFunction._f, k)


XgFunction = _LazyFunction()

from ._batch import (Batch, Graph, autotune, autotune_adjoint, autotune_batch,  # noqa: E402
                     autotune_batch_precompile, autotune_precompile, capture_eval, capture_rollout)
