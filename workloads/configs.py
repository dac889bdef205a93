"""The five workloads: programs, instance counts, dtypes and input seeds.

1. random scalar DAG: 8 inputs ~U(-1,1), 4 outputs, 200 drawn ops, N=1,000,
   fp64, forward;
2. planar 7-link pendulum, one RK4 step (dt=1e-3), N=16,384, fp64 and fp32;
3. closed-form cart-pole MPC (T=20, 3 penalty-SQP iterations, fixed-pattern
   LDL^T), N=4,096, fp64;
4. gradient of ||s'||^2 w.r.t. s for workload 2, N=65,536, fp64 and fp32;
5. one persistent launch of three random DAGs (1e3/1e4/1e5 ops, 16/32/64
   inputs, N=65,536/8,192/512, fp32) plus workload 3 at N=2,048 (fp64).

Program seeds and input seeds are fixed here; programs are cached as files
under a cache directory so both evaluators read identical bytes.
"""

from __future__ import annotations

import os
from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from . import inputs
from .ldl import SIZES as LDL_SIZES, ldl_solve, spd_inputs
from .mpc import cartpole_mpc
from .pendulum import pendulum
from .quadcopter import quad_closed_loop, quad_initial, quad_params
from .rdag import rdag


@dataclass
class Item:
    key: str
    build: Callable
    n: int
    dtype: str
    make_inputs: Callable  # (n) -> list of (nnz, n) float64 arrays
    extra: dict = field(default_factory=dict)


def _pend_in(seed):
    return lambda n: [inputs.pendulum_state(seed, 7, n)]


ITEMS = {
    "rdag200": Item("rdag200", lambda: rdag(1, 8, 200), 1000, "f64",
                    lambda n: [inputs.uniform(101, 8, n)]),
    "pend7": Item("pend7", lambda: pendulum(7), 16384, "f64", _pend_in(102)),
    "pend7_f32": Item("pend7_f32", lambda: pendulum(7, dtype="f32"), 16384, "f32", _pend_in(102)),
    "mpc": Item("mpc", lambda: cartpole_mpc(), 4096, "f64",
                lambda n: [inputs.cartpole_state(103, n)]),
    "pend7_grad": Item("pend7_grad", lambda: pendulum(7), 65536, "f64", _pend_in(104)),
    "pend7_grad_f32": Item("pend7_grad_f32", lambda: pendulum(7, dtype="f32"), 65536, "f32",
                           _pend_in(104)),
    "rdag1e3": Item("rdag1e3", lambda: rdag(51, 16, 1000, dtype="f32"), 65536, "f32",
                    lambda n: [inputs.uniform(151, 16, n)]),
    "rdag1e4": Item("rdag1e4", lambda: rdag(52, 32, 10000, dtype="f32"), 8192, "f32",
                    lambda n: [inputs.uniform(152, 32, n)]),
    "rdag1e5": Item("rdag1e5", lambda: rdag(53, 64, 100000, dtype="f32"), 512, "f32",
                    lambda n: [inputs.uniform(153, 64, n)]),
    "mpc_mixed": Item("mpc_mixed", lambda: cartpole_mpc(precision="mixed"), 4096, "f64",
                      lambda n: [inputs.cartpole_state(103, n)]),
    "mpc_b": Item("mpc_b", lambda: cartpole_mpc(), 2048, "f64",
                  lambda n: [inputs.cartpole_state(105, n)]),
}

# The iteration-count sweep of the closed-form MPC: M = 1 is the real-time
# iteration variant (one SQP step from the constant initial guess); M = 3 is
# the "mpc" item above.
for _m in (1, 2, 4, 5):
    ITEMS[f"mpc_m{_m}"] = Item(f"mpc_m{_m}", (lambda m: lambda: cartpole_mpc(iters=m))(_m), 4096,
                               "f64", lambda n: [inputs.cartpole_state(103, n)])
MPC_SWEEP = ["mpc_m1", "mpc_m2", "mpc", "mpc_m4", "mpc_m5"]

# The paper's benchmark family: dense LDL^T solves of SPD systems whose
# operation counts grow about 10x per size, swept over batch sizes.
for _i, _n in enumerate(LDL_SIZES):
    ITEMS[f"ldl{_n}"] = Item(f"ldl{_n}", (lambda n: lambda: ldl_solve(n))(_n), 10000, "f64",
                             (lambda n, seed: lambda cnt: spd_inputs(seed, n, cnt))(_n, 161 + _i))
LDL_SWEEP = [f"ldl{_n}" for _n in LDL_SIZES]

# The quadcopter closed-loop LQR step (state, parameters) -> state, rolled out
# for 10,000 environments.
ITEMS["quad"] = Item("quad", lambda: quad_closed_loop(), 10000, "f64",
                     lambda n: [quad_initial(201, n), quad_params(202, n)])
LDL_BATCHES = (10, 100, 1000, 10000, 100000)

CONFIGS = {
    1: ["rdag200"],
    2: ["pend7", "pend7_f32"],
    3: ["mpc"],
    4: ["pend7_grad", "pend7_grad_f32"],
    5: ["rdag1e3", "rdag1e4", "rdag1e5", "mpc_b"],
}


def cache_dir() -> str:
    d = os.environ.get("XG_WORKLOAD_DIR") or os.path.join(
        os.path.dirname(os.path.abspath(__file__)), "_programs")
    os.makedirs(d, exist_ok=True)
    return d


def _source_tag() -> str:
    """Short hash of the builder sources, so a stale cached file is never used."""
    import hashlib
    h = hashlib.sha1()
    here = os.path.dirname(os.path.abspath(__file__))
    for f in ("tracer.py", "pendulum.py", "mpc.py", "rdag.py", "ldl.py", "quadcopter.py",
              "configs.py"):
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:10]


def program_path(key: str) -> str:
    """Path of the item's program file, building it on first use."""
    path = os.path.join(cache_dir(), f"{key}-{_source_tag()}.xgp")
    if not os.path.exists(path):
        prog = ITEMS[key].build()
        tmp = f"{path}.tmp{os.getpid()}"
        prog.save(tmp)
        os.replace(tmp, path)
    return path


def program(key: str):
    return ITEMS[key].build()


def item_inputs(key: str, n: int | None = None) -> list[np.ndarray]:
    it = ITEMS[key]
    return it.make_inputs(it.n if n is None else n)
