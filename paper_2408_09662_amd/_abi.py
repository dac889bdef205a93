"""ctypes declarations mirroring include/xg.h."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxg.so")

XG_F32, XG_F64 = 32, 64

# Opcode names in the order of the xg_op enum of include/xg.h
OPS = ["INPUT", "OUTPUT", "CONST", "ASSIGN", "ADD", "SUB", "MUL", "DIV", "NEG", "SQ", "SQRT",
       "EXP", "LOG", "SIN", "COS", "TAN", "TANH", "ATAN", "FABS", "FMIN", "FMAX", "LT", "LE",
       "POW", "ATAN2"]
OP_ID = {k: i for i, k in enumerate(OPS)}

STATUS = {0: "XG_OK", -1: "XG_EINVAL", -2: "XG_EALIAS", -3: "XG_ENOMEM", -4: "XG_ECOMPILE",
          -5: "XG_EDEVICE", -6: "XG_EUNSUPPORTED"}


class XgError(RuntimeError):
    def __init__(self, msg, status=None):
        super().__init__(msg)
        self.status = status


class ProgramDesc(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("nnz_in", ctypes.c_void_p),
                ("n_out", ctypes.c_int32), ("nnz_out", ctypes.c_void_p),
                ("n_work", ctypes.c_int32), ("n_instr", ctypes.c_int64),
                ("instr", ctypes.c_void_p), ("n_const", ctypes.c_int32),
                ("consts", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("prec", ctypes.c_void_p)]

    def __init__(self, **kw):
        for k in ("nnz_in", "nnz_out"):
            if k in kw and not isinstance(kw[k], (int, ctypes.c_void_p)) and kw[k] is not None:
                kw[k] = ctypes.cast(kw[k], ctypes.c_void_p)
        super().__init__(**kw)


OPTION_FIELDS = ["block", "ipt", "chunk_ops", "reg_budget", "lds_slots", "strict", "eager",
                 "adj_seg_ops", "verbose", "prefetch", "waves", "inline_math", "adj_fanout",
                 "coop_phase"]


class Options(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in OPTION_FIELDS]


def make_options(d: dict) -> Options:
    unknown = set(d) - set(OPTION_FIELDS)
    if unknown:
        raise XgError(f"unknown options {sorted(unknown)}")
    o = Options()
    for k, v in d.items():
        setattr(o, k, int(v))
    return o


class Info(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_ops", ctypes.c_int64),
                ("max_live", ctypes.c_int64), ("n_chunks", ctypes.c_int32),
                ("n_ws_slots", ctypes.c_int32), ("n_lds_slots", ctypes.c_int32),
                ("n_spills", ctypes.c_int32), ("compile_ms", ctypes.c_double),
                ("cache_hits", ctypes.c_int32), ("vgprs", ctypes.c_int32),
                ("code_hash", ctypes.c_uint64), ("lds_bytes", ctypes.c_int32),
                ("scratch_bytes", ctypes.c_int32)]


class BatchArgs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d_in", ctypes.c_void_p), ("ld_in", ctypes.c_void_p),
                ("d_out", ctypes.c_void_p), ("ld_out", ctypes.c_void_p)]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SIGS = {
    "xg_program_load": ([_P, _P, _P], _I32),
    "xg_program_free": ([_P], None),
    "xg_program_info": ([_P, _I32, _P], _I32),
    "xg_workspace_bytes": ([_P, _I64, _I32, _P], _I32),
    "xg_compile": ([_P, _I32], _I32),
    "xg_precompile": ([_P, _I32], _I32),
    "xg_eval": ([_P, _I64, _P, _P, _P, _P, _P, _P], _I32),
    "xg_eval_adjoint": ([_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P], _I32),
    "xg_eval_adjoint_noalloc": ([_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P], _I32),
    "xg_batch_create": ([_P, _I32, _P, _P], _I32),
    "xg_batch_free": ([_P], None),
    "xg_batch_workspace_bytes": ([_P, _P, _P], _I32),
    "xg_batch_eval": ([_P, _P, _P, _P], _I32),
    "xg_graph_capture_eval": ([_P, _I64, _P, _P, _P, _P, _P, _P, _P], _I32),
    "xg_graph_capture_batch": ([_P, _P, _P, _P, _P], _I32),
    "xg_graph_launch": ([_P, _P], _I32),
    "xg_graph_free": ([_P], None),
    "xg_autotune": ([_P, _I64, _P, _P, _P, _P, _P, ctypes.c_size_t, _P, _P], _I32),
    "xg_autotune_precompile": ([_P, _I64, _I32], _I32),
    "xg_batch_autotune": ([_P, _I32, _P, _P, ctypes.c_size_t, _P, _P, ctypes.POINTER(_I32)], _I32),
    "xg_batch_autotune_workspace_bytes": ([_P, _I32, _P, ctypes.POINTER(ctypes.c_size_t)], _I32),
    "xg_batch_autotune_precompile": ([_P, _I32, _P], _I32),
    "xg_autotune_adjoint": ([_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P, _P], _I32),
    "xg_graph_capture_rollout": ([_P, _I64, _I32, _P, _P, _I64, _P, _P, _P, _P, ctypes.c_void_p], _I32),
    "xg_program_options": ([_P, _I32, ctypes.c_void_p], _I32),
    "xg_autotune_workspace_bytes": ([_P, _I64, _I32, ctypes.POINTER(ctypes.c_size_t)], _I32),
    "xg_last_error": ([], ctypes.c_char_p),
    "xg_version": ([], ctypes.c_char_p),
}


def lib():
    """The loaded native library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2408_09662_amd.build` (no fallback exists)")
        # torch first: libxg.so then binds the HIP runtime torch has loaded
        # (torch ships its own copy), so the process holds one HIP runtime
        # and torch's streams and allocations are valid in library calls
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != 0:
        msg = lib().xg_last_error().decode(errors="replace")
        raise XgError(f"{STATUS.get(status, status)}: {msg}", status)
