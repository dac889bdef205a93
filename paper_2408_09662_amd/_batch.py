"""Persistent multi-program batches, HIP-graph replay and the autotuner
(binding: argument marshalling only)."""

from __future__ import annotations

import ctypes

from . import _abi
from ._abi import lib


def _torch():
    import torch
    return torch


class Batch:
    """Several programs evaluated in ONE persistent launch.

    The programs (paper_2408_09662_amd.Program) are borrowed and must outlive
    the batch; they must share the block and ipt options."""

    def __init__(self, programs, verbose: bool = False):
        from . import _ptrs  # noqa: F401  (binding helpers)
        self.programs = list(programs)
        arr = (ctypes.c_void_p * len(self.programs))(*[p._h.value for p in self.programs])
        opts = _abi.make_options({"verbose": int(verbose)})
        h = ctypes.c_void_p()
        _abi.check(lib().xg_batch_create(arr, len(self.programs), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._ws = None

    @classmethod
    def _adopt(cls, programs, handle, block):
        """Wrap a batch the library made (it owns its own program copies;
        `programs` only supply argument shapes and dtypes)."""
        b = cls.__new__(cls)
        b.programs = list(programs)
        b._h = handle
        b._ws = None
        b.block = block
        return b

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _abi is not None and _abi._lib is not None:
            _abi._lib.xg_batch_free(h)  # (module globals may be gone at interpreter exit)
            self._h = None

    def workspace_bytes(self, ns) -> int:
        arr = (ctypes.c_int64 * len(ns))(*ns)
        b = ctypes.c_size_t()
        _abi.check(lib().xg_batch_workspace_bytes(self._h, arr, ctypes.byref(b)))
        return b.value

    def workspace(self, ns):
        torch = _torch()
        nb = self.workspace_bytes(ns)
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        return self._ws

    def _args(self, inputs, outputs):
        from . import _ptrs
        k = len(self.programs)
        if len(inputs) != k or len(outputs) != k:
            raise _abi.XgError(f"a batch of {k} programs needs {k} input and {k} output lists")
        A = (_abi.BatchArgs * k)()
        keep = []
        ns = []
        for i, p in enumerate(self.programs):
            n = p._n_of(inputs[i], None)
            ns.append(n)
            pi, li = _ptrs(inputs[i], n, p.torch_dtype, p.nnz_in, f"program {i} input")
            po, lo = _ptrs(outputs[i], n, p.torch_dtype, p.nnz_out, f"program {i} output")
            keep += [pi, li, po, lo]
            A[i].n = n
            A[i].d_in = ctypes.cast(pi, ctypes.c_void_p)
            A[i].ld_in = ctypes.cast(li, ctypes.c_void_p)
            A[i].d_out = ctypes.cast(po, ctypes.c_void_p)
            A[i].ld_out = ctypes.cast(lo, ctypes.c_void_p)
        return A, ns, keep

    def eval(self, inputs, outputs=None, stream=None, workspace=None):
        """inputs[k]: list of (nnz, N_k) tensors of program k.  Returns outputs."""
        from . import _stream_handle
        if outputs is None:
            outputs = [p.alloc_outputs(p._n_of(inputs[i], None)) for i, p in enumerate(self.programs)]
        A, ns, keep = self._args(inputs, outputs)
        ws = workspace if workspace is not None else self.workspace(ns)
        _abi.check(lib().xg_batch_eval(self._h, A, ctypes.c_void_p(ws.data_ptr()),
                                       _stream_handle(stream)))
        del keep
        return outputs

    def capture(self, inputs, outputs, stream, workspace=None) -> "Graph":
        from . import _stream_handle
        A, ns, keep = self._args(inputs, outputs)
        ws = workspace if workspace is not None else self.workspace(ns)
        g = ctypes.c_void_p()
        _abi.check(lib().xg_graph_capture_batch(self._h, A, ctypes.c_void_p(ws.data_ptr()),
                                                _stream_handle(stream), ctypes.byref(g)))
        # the graph launches this batch's kernel: keep the batch (and through
        # it its programs) alive as long as the graph
        return Graph(g, keep=(self, inputs, outputs, ws, keep))


class Graph:
    """A captured launch sequence; replay with launch(stream).  The program
    or batch it launches and the buffers it was captured with are kept alive
    (and must not move) as long as the graph.  While a graph of a program
    exists, autotuning that program is refused by the library."""

    def __init__(self, handle, keep=None):
        self._h = handle
        self._keep = keep

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _abi is not None and _abi._lib is not None:
            _abi._lib.xg_graph_free(h)  # (module globals may be gone at interpreter exit)
            self._h = None

    def launch(self, stream=None):
        from . import _stream_handle
        _abi.check(lib().xg_graph_launch(self._h, _stream_handle(stream)))


def capture_eval(prog, inputs, outputs, stream, workspace=None) -> Graph:
    """Capture prog.eval(inputs -> outputs) on a non-default stream."""
    from . import _ptrs, _stream_handle
    n = prog._n_of(inputs, None)
    pi, li = _ptrs(inputs, n, prog.torch_dtype, prog.nnz_in, "input")
    po, lo = _ptrs(outputs, n, prog.torch_dtype, prog.nnz_out, "output")
    ws = workspace if workspace is not None else prog.workspace(n, 0)
    g = ctypes.c_void_p()
    _abi.check(lib().xg_graph_capture_eval(prog._h, n, pi, li, po, lo,
                                           ctypes.c_void_p(ws.data_ptr() if ws is not None else 0),
                                           _stream_handle(stream), ctypes.byref(g)))
    return Graph(g, keep=(prog, inputs, outputs, ws, pi, li, po, lo))


def capture_rollout(prog, state0, state1, others, steps: int, stream, workspace=None) -> Graph:
    """Capture `steps` closed-loop evaluations state <- prog(state, *others)
    ping-ponging between state0 and state1 ((nnz, N) tensors of the same
    pitch); after a replay the state is in state0 if steps is even, else in
    state1."""
    from . import _ptrs, _stream_handle
    n = state0.shape[1]
    if state1.shape != state0.shape or state1.stride() != state0.stride():
        raise _abi.XgError("state buffers must have the same shape and pitch")
    if len(prog.nnz_out) != 1 or prog.nnz_out[0] != prog.nnz_in[0]:
        raise _abi.XgError("rollout needs a program whose only output has the shape of its first input")
    pi, li = _ptrs([state0] + list(others), n, prog.torch_dtype, prog.nnz_in, "input")
    ws = workspace if workspace is not None else prog.workspace(n, 0)
    g = ctypes.c_void_p()
    _abi.check(lib().xg_graph_capture_rollout(
        prog._h, n, steps, ctypes.c_void_p(state0.data_ptr()), ctypes.c_void_p(state1.data_ptr()),
        li[0], pi, li, ctypes.c_void_p(ws.data_ptr() if ws is not None else 0),
        _stream_handle(stream), ctypes.byref(g)))
    return Graph(g, keep=(prog, state0, state1, others, ws, pi, li))


def autotune_precompile(prog, n: int, mode: int = 0) -> None:
    """Compile every candidate autotune() (mode 0) or autotune_adjoint()
    (mode 1 or 2) would time for n instances (no GPU)."""
    _abi.check(lib().xg_autotune_precompile(prog._h, n, mode))


def autotune(prog, inputs, outputs=None, stream=None) -> dict:
    """Time plan candidates for this instance count and adopt the fastest
    (cached on disk).  Returns the chosen options."""
    from . import _ptrs, _stream_handle
    torch = _torch()
    n = prog._n_of(inputs, None)
    if outputs is None:
        outputs = prog.alloc_outputs(n)
    pi, li = _ptrs(inputs, n, prog.torch_dtype, prog.nnz_in, "input")
    po, lo = _ptrs(outputs, n, prog.torch_dtype, prog.nnz_out, "output")
    b = ctypes.c_size_t()
    _abi.check(lib().xg_autotune_workspace_bytes(prog._h, n, 0, ctypes.byref(b)))
    nb = max(b.value, 256)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    chosen = _abi.Options()
    _abi.check(lib().xg_autotune(prog._h, n, pi, li, po, lo, ctypes.c_void_p(ws.data_ptr()), nb,
                                 _stream_handle(stream), ctypes.byref(chosen)))
    prog._ws = {}
    return {f: getattr(chosen, f) for f in _abi.OPTION_FIELDS}


def autotune_adjoint(prog, inputs, seeds, fused: bool = True, stream=None) -> dict:
    """Time adjoint plan candidates for this instance count on the fused
    forward+adjoint kernel (fused=True) or the gradient-only one, and adopt
    the fastest for both adjoint modes (cached on disk).  Returns the chosen
    options."""
    from . import _ptrs, _stream_handle
    torch = _torch()
    n = prog._n_of(inputs, None)
    mode = 2 if fused else 1
    grads = [torch.empty((k, n), dtype=prog.torch_dtype, device="cuda") for k in prog.nnz_in]
    pi, li = _ptrs(inputs, n, prog.torch_dtype, prog.nnz_in, "input")
    ps, ls = _ptrs(seeds, n, prog.torch_dtype, prog.nnz_out, "seed")
    pg, lg = _ptrs(grads, n, prog.torch_dtype, prog.nnz_in, "gradient")
    outs = prog.alloc_outputs(n) if fused else None  # held until the call returns
    if fused:
        po, lo = _ptrs(outs, n, prog.torch_dtype, prog.nnz_out, "output")
    else:
        po, lo = None, None
    b = ctypes.c_size_t()
    _abi.check(lib().xg_autotune_workspace_bytes(prog._h, n, mode, ctypes.byref(b)))
    nb = max(b.value, 256)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    chosen = _abi.Options()
    _abi.check(lib().xg_autotune_adjoint(prog._h, n, pi, li, ps, ls, po, lo, pg, lg,
                                         ctypes.c_void_p(ws.data_ptr()), nb, _stream_handle(stream),
                                         ctypes.byref(chosen)))
    prog._ws = {}
    return {f: getattr(chosen, f) for f in _abi.OPTION_FIELDS}


def autotune_batch_precompile(programs, ns) -> None:
    """Compile every candidate autotune_batch() would time (no GPU)."""
    k = len(programs)
    arr = (ctypes.c_void_p * k)(*[p._h.value for p in programs])
    na = (ctypes.c_int64 * k)(*ns)
    _abi.check(lib().xg_batch_autotune_precompile(arr, k, na))


def autotune_batch(programs, inputs, outputs=None, stream=None) -> "Batch":
    """Time persistent-launch arrangements of these programs (workgroup size,
    cooperative tiles for wide programs with few tiles) on the given inputs
    and return the fastest as a new Batch (the choice is cached on disk).
    The programs are not changed; the batch holds its own tuned copies."""
    from . import _stream_handle
    torch = _torch()
    k = len(programs)
    if outputs is None:
        outputs = [p.alloc_outputs(p._n_of(inputs[i], None)) for i, p in enumerate(programs)]
    probe = Batch.__new__(Batch)
    probe.programs = list(programs)
    A, ns, keep = Batch._args(probe, inputs, outputs)
    arr = (ctypes.c_void_p * k)(*[p._h.value for p in programs])
    na = (ctypes.c_int64 * k)(*ns)
    b = ctypes.c_size_t()
    _abi.check(lib().xg_batch_autotune_workspace_bytes(arr, k, na, ctypes.byref(b)))
    ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    block = ctypes.c_int32()
    _abi.check(lib().xg_batch_autotune(arr, k, A, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       _stream_handle(stream), ctypes.byref(h), ctypes.byref(block)))
    del keep
    return Batch._adopt(programs, h, block.value)

