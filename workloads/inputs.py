"""Seeded synthetic inputs, structure-of-arrays, instance-fastest.

Every input argument is an array of shape (nnz, N) (element e of instance n
at [e, n]), float64 little-endian.  fp32 runs use the same draws rounded
once to float32.  Distributions follow the workload descriptions:

* random DAGs:   x ~ U(-1, 1);
* pendulum:      q_i ~ U(-pi, pi), qdot_i ~ N(0, 1);
* cart-pole MPC: xbar_0 ~ U([-1,1] x [-pi,pi] x [-1,1] x [-1,1]);
* adjoint seeds: drawn by the caller (the pendulum loss uses ybar = 2 s').
"""

from __future__ import annotations

import numpy as np


def uniform(seed: int, nnz: int, n: int, lo=-1.0, hi=1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(lo, hi, size=(nnz, n)))


def pendulum_state(seed: int, n_links: int, n: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    q = rng.uniform(-np.pi, np.pi, size=(n_links, n))
    qd = rng.standard_normal(size=(n_links, n))
    return np.ascontiguousarray(np.concatenate([q, qd], axis=0))


def cartpole_state(seed: int, n: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    lo = np.array([-1.0, -np.pi, -1.0, -1.0])[:, None]
    hi = np.array([1.0, np.pi, 1.0, 1.0])[:, None]
    return np.ascontiguousarray(lo + (hi - lo) * rng.random(size=(4, n)))


def to_dtype(x: np.ndarray, dtype: str) -> np.ndarray:
    """Round once to the program's dtype (f32) and return float64 storage
    of the rounded values, or the float32 array itself if asked."""
    if dtype == "f64":
        return x
    if dtype == "f32":
        return x.astype(np.float32)
    raise ValueError(dtype)
