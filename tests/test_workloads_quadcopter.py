"""Pins of the quadcopter closed-loop LQR step as evaluated by the oracle.

(i)   The doubling iteration's Riccati solution S and the gain K equal
      SciPy's discrete algebraic Riccati solver (a library routine) applied
      to A, B derived here by hand from the step equations.
(ii)  Hover at the origin is a fixed point.
(iii) Thrusts stay inside [0, u_max]; far from hover they saturate.
(iv)  Small perturbations decay under the closed loop (stabilising gain).
(v)   Long double vs double agree to 1e-13 (the 1e-12 gate is meaningful).
"""

import numpy as np
import pytest
import scipy.linalg as sl

from oracle.pyoracle import evaluate_program
from workloads.quadcopter import GRAV, quad_closed_loop, quad_initial, quad_params

DT = 0.01


def hand_linearisation(m, inertia, arm, dt=DT):
    A = np.eye(6)
    A[0, 3] = A[1, 4] = A[2, 5] = dt
    A[3, 2] = -dt * GRAV
    A[0, 2] = -dt * dt * GRAV
    B = np.zeros((6, 2))
    B[4, :] = dt / m
    B[1, :] = dt * dt / m
    B[5, 0], B[5, 1] = dt * arm / inertia, -dt * arm / inertia
    B[2, 0], B[2, 1] = dt * dt * arm / inertia, -dt * dt * arm / inertia
    return A, B


@pytest.fixture(scope="module")
def debug_prog():
    return quad_closed_loop(outputs="debug")


def test_riccati_and_gain_match_scipy(debug_prog, tmp_path):
    n = 32
    th = quad_params(11, n)
    z = quad_initial(12, n)
    _, u, K, S = evaluate_program(debug_prog, [z, th], tmpdir=tmp_path)
    for i in range(n):
        m, inertia, arm = th[0, i], th[1, i], th[2, i]
        A, B = hand_linearisation(m, inertia, arm)
        Q, R = np.diag(th[4:10, i]), np.diag(th[10:12, i])
        X = sl.solve_discrete_are(A, B, Q, R)
        Kr = np.linalg.solve(R + B.T @ X @ B, B.T @ X @ A)
        assert np.max(np.abs(S[:, i].reshape(6, 6) - X)) <= 1e-9 * np.max(np.abs(X))
        assert np.max(np.abs(K[:, i].reshape(2, 6) - Kr)) <= 1e-8 * np.max(np.abs(Kr))


def test_hover_is_a_fixed_point(tmp_path):
    n = 16
    th = quad_params(13, n)
    z1 = evaluate_program(quad_closed_loop(), [np.zeros((6, n)), th], tmpdir=tmp_path)[0]
    assert np.max(np.abs(z1)) <= 1e-14


def test_thrusts_clamped_and_saturating(debug_prog, tmp_path):
    n = 64
    th = quad_params(14, n)
    z = quad_initial(15, n) * 10.0  # far from hover
    _, u, _, _ = evaluate_program(debug_prog, [z, th], tmpdir=tmp_path)
    assert np.all(u >= 0.0) and np.all(u <= th[3])
    assert np.mean((u == 0.0) | (u == th[3])) > 0.5


def test_small_perturbations_decay(tmp_path):
    n = 16
    th = quad_params(16, n)
    z = quad_initial(17, n) * 0.05
    prog = quad_closed_loop()
    from oracle.pyoracle import Program
    path = tmp_path / "q.xgp"
    prog.save(path)
    o = Program(path)
    norms = [np.max(np.abs(z))]
    for _ in range(400):
        z = o.evaluate([z, th])[0]
    norms.append(np.max(np.abs(z)))
    assert norms[1] < 0.2 * norms[0], norms


def test_inherent_sensitivity(tmp_path):
    n = 512
    th = quad_params(18, n)
    z = quad_initial(19, n)
    prog = quad_closed_loop()
    y64 = evaluate_program(prog, [z, th], 64, tmpdir=tmp_path)[0]
    y80 = evaluate_program(prog, [z, th], 80, tmpdir=tmp_path)[0]
    sc = np.sqrt(np.mean(y80 ** 2, axis=1, keepdims=True))
    assert (np.abs(y64 - y80) / np.maximum(np.abs(y80), sc)).max() <= 1e-13
