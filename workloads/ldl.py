"""Dense LDL^T solutions of symmetric positive definite systems.

The paper's benchmark family (section "Benchmarking"): functions that return
the solution of a positive definite linear system through an LDL^T
decomposition, in five sizes whose operation counts are about an order of
magnitude apart, evaluated over a sweep of batch sizes.

ldl_solve(n): inputs  A (the n(n+1)/2 entries of its lower triangle, row by
row: A[0,0], A[1,0], A[1,1], A[2,0], ...) and b (n); output x = A^{-1} b.
The factorisation is the textbook one without pivoting:

    D_j    = A_jj - sum_{k<j} L_jk^2 D_k
    L_ij   = (A_ij - sum_{k<j} L_ik L_jk D_k) / D_j        (i > j)

then L y = b, z = y / D, L^T x = z.  Every pivot D_j is positive for an SPD
matrix, so no pivoting is needed.
"""

from __future__ import annotations

import numpy as np

from .tracer import Graph

# matrix sizes of the family: operation counts about 10x apart
SIZES = (4, 10, 22, 48, 104)


def tri_index(i: int, j: int) -> int:
    """Position of A[i, j] (i >= j) in the packed lower triangle."""
    return i * (i + 1) // 2 + j


def ldl_solve(n: int, dtype: str = "f64", reuse_slots: bool = True):
    g = Graph(f"ldl_solve_{n}", dtype)
    A = g.input(n * (n + 1) // 2)
    b = g.input(n)
    a = lambda i, j: A[tri_index(i, j)]  # noqa: E731
    L = {}
    D = []
    for j in range(n):
        # LD_k = L_jk D_k, reused by the whole column j
        LD = [L[(j, k)] * D[k] for k in range(j)]
        d = a(j, j)
        for k in range(j):
            d = d - LD[k] * L[(j, k)]
        D.append(d)
        for i in range(j + 1, n):
            s = a(i, j)
            for k in range(j):
                s = s - L[(i, k)] * LD[k]
            L[(i, j)] = s / d
    y = []
    for i in range(n):
        s = b[i]
        for k in range(i):
            s = s - L[(i, k)] * y[k]
        y.append(s)
    z = [y[i] / D[i] for i in range(n)]
    x = [None] * n
    for i in reversed(range(n)):
        s = z[i]
        for k in range(i + 1, n):
            s = s - L[(k, i)] * x[k]
        x[i] = s
    return g.program([x], reuse_slots=reuse_slots)


def spd_inputs(seed: int, n: int, count: int):
    """Seeded, strictly diagonally dominant SPD systems (so positive definite
    by Gershgorin): off-diagonal A_ij ~ U(-1, 1), A_ii = n + U(0, 1);
    b ~ N(0, 1).  Returns [A packed lower triangle (n(n+1)/2, count),
    b (n, count)]."""
    rng = np.random.default_rng(seed)
    m = n * (n + 1) // 2
    A = rng.uniform(-1.0, 1.0, size=(m, count))
    for i in range(n):
        A[tri_index(i, i)] = n + rng.random(count)
    b = rng.standard_normal(size=(n, count))
    return [np.ascontiguousarray(A), np.ascontiguousarray(b)]


def dense(Ap: np.ndarray, n: int, inst: int) -> np.ndarray:
    """The full symmetric matrix of instance `inst` from its packed triangle."""
    M = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            M[i, j] = M[j, i] = Ap[tri_index(i, j), inst]
    return M
