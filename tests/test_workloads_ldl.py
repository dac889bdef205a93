"""Pins of the LDL^T-solve family (the paper's benchmark functions) as
evaluated by the oracle: the result solves A x = b (checked against LAPACK
through numpy on the dense matrix), and long double vs double agree to
1e-13 (so a 1e-12 parity gate is meaningful)."""

import numpy as np
import pytest

from oracle.pyoracle import evaluate_program
from workloads.ldl import SIZES, dense, ldl_solve, spd_inputs


@pytest.mark.parametrize("n", SIZES[:4])
def test_solution_matches_lapack(n, tmp_path):
    cnt = 40
    A, b = spd_inputs(7 + n, n, cnt)
    x = evaluate_program(ldl_solve(n), [A, b], tmpdir=tmp_path)[0]
    for inst in range(cnt):
        M = dense(A, n, inst)
        ref = np.linalg.solve(M, b[:, inst])
        assert np.max(np.abs(x[:, inst] - ref)) <= 1e-13 * np.max(np.abs(ref)) * n
        r = M @ x[:, inst] - b[:, inst]
        assert np.max(np.abs(r)) <= 1e-13 * n * np.max(np.abs(b[:, inst]))


def test_largest_size_solves_its_system(tmp_path):
    n = SIZES[-1]
    A, b = spd_inputs(3, n, 3)
    x = evaluate_program(ldl_solve(n), [A, b], tmpdir=tmp_path)[0]
    for inst in range(3):
        ref = np.linalg.solve(dense(A, n, inst), b[:, inst])
        assert np.max(np.abs(x[:, inst] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_identity_and_diagonal_special_cases(tmp_path):
    """A = diag(d): x = b / d exactly (no off-diagonal terms enter)."""
    n = 10
    A, b = spd_inputs(1, n, 8)
    A[:] = 0.0
    d = np.arange(1, n + 1, dtype=float)
    for i in range(n):
        A[i * (i + 1) // 2 + i] = d[i]
    x = evaluate_program(ldl_solve(n), [A, b], tmpdir=tmp_path)[0]
    assert np.array_equal(x, b / d[:, None])


def test_operation_counts_grow_tenfold():
    counts = [ldl_solve(n).n_arith() for n in SIZES[:4]]
    for a, c in zip(counts, counts[1:]):
        assert 6 < c / a < 14, counts


@pytest.mark.parametrize("n", SIZES[:4])
def test_inherent_sensitivity(n, tmp_path):
    A, b = spd_inputs(161, n, 256)
    prog = ldl_solve(n)
    y64 = evaluate_program(prog, [A, b], 64, tmpdir=tmp_path)[0]
    y80 = evaluate_program(prog, [A, b], 80, tmpdir=tmp_path)[0]
    sc = np.sqrt(np.mean(y80 ** 2, axis=1, keepdims=True))
    assert (np.abs(y64 - y80) / np.maximum(np.abs(y80), sc)).max() <= 1e-13
