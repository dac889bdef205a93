"""Pins of the closed-form MPC program as evaluated by the oracle.

(i)   Closed form: with linear dynamics and no inequality penalty, one SQP
      iteration solves the equality-constrained QP exactly, so its result is
      the finite-horizon LQR trajectory from a backward Riccati recursion
      (computed here in long double); further iterations leave it unchanged.
(ii)  The KKT solve: the program's solution satisfies K v = rhs for a KKT
      matrix K assembled here, independently, from the program's own
      Jacobians and Hessian diagonal, and equals long-double Gaussian
      elimination with partial pivoting.
(iii) The pivot signs of the chosen unknown order: every x/u pivot > 0,
      every multiplier pivot < 0 (so no pivoting is needed).
(iv)  The cart-pole RK4 step conserves energy and horizontal momentum with
      F = 0 to fifth local order.
(v)   The dynamics defect falls over the SQP iterations near upright.
(vi)  Inherent sensitivity: long double vs double <= 1e-11.
"""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from workloads import inputs
from workloads.mpc import CartPole, Linear, NX, cartpole_mpc, cartpole_step, kkt_index

Qd = np.array([1.0, 1.0, 0.1, 0.1])
QT_SCALE = 10.0
R = 0.1


def run(prog, xs, tmp_path, scalar=64, name="m"):
    path = tmp_path / f"{name}.xgp"
    prog.save(path)
    return OProg(path).evaluate(xs, scalar, threads=4)


def _lin_AB():
    dt = 0.02
    Ac = np.array([[0, 0, 1, 0], [0, 0, 0, 1], [0, -0.98, 0, 0], [0, 21.6, 0, 0]], dtype=float)
    A = np.eye(4) + dt * Ac + 0.5 * dt * dt * Ac @ Ac
    B = dt * np.array([[0.0], [0.0], [1.0], [-2.0]])
    return A, B


def _riccati_rollout(A, B, x0, T):
    ld = np.longdouble
    A = A.astype(ld)
    B = B.astype(ld)
    Q = np.diag(Qd).astype(ld)
    P = QT_SCALE * Q
    Ks = [None] * T
    for k in reversed(range(T)):
        S = ld(R) + (B.T @ P @ B)[0, 0]
        K = (B.T @ P @ A) / S
        Ks[k] = K
        P = Q + A.T @ P @ (A - B @ K)
    xs = [x0.astype(ld)]
    us = []
    for k in range(T):
        u = -(Ks[k] @ xs[-1])
        us.append(u[0])
        xs.append(A @ xs[-1] + B[:, 0] * u[0])
    return np.concatenate([np.concatenate(xs), np.array(us)])


@pytest.mark.parametrize("iters", [1, 3])
def test_linear_unpenalised_equals_riccati_lqr(tmp_path, iters):
    A, B = _lin_AB()
    T = 20
    prog = cartpole_mpc(T=T, iters=iters, dyn=Linear(A, B), penalty=False)
    x0 = inputs.cartpole_state(33, 40)
    z = run(prog, [x0], tmp_path, name=f"lqr{iters}")[0]
    for i in range(x0.shape[1]):
        ref = _riccati_rollout(A, B, x0[:, i], T).astype(np.float64)
        sc = np.max(np.abs(ref))
        assert np.max(np.abs(z[:, i] - ref)) <= 1e-12 * sc, i


def _assemble(T, A, B, huu):
    ix, il, iu, n = kkt_index(T)
    ld = np.longdouble
    K = np.zeros((n, n), dtype=ld)
    for k in range(T + 1):
        Qk = Qd * (QT_SCALE if k == T else 1.0)
        for i in range(NX):
            K[ix[k] + i, ix[k] + i] = Qk[i]
            K[il[k] + i, ix[k] + i] = K[ix[k] + i, il[k] + i] = 1.0
            if k > 0:
                for j in range(NX):
                    K[il[k] + i, ix[k - 1] + j] = K[ix[k - 1] + j, il[k] + i] = -A[k - 1, i, j]
                K[il[k] + i, iu[k - 1]] = K[iu[k - 1], il[k] + i] = -B[k - 1, i]
        if k < T:
            K[iu[k], iu[k]] = huu[k]
    return K


def _solve_ld(A, b):
    A = A.copy()
    b = b.copy()
    n = len(b)
    for k in range(n):
        p = k + int(np.argmax(np.abs(A[k:, k])))
        A[[k, p]] = A[[p, k]]
        b[[k, p]] = b[[p, k]]
        f = A[k + 1:, k] / A[k, k]
        A[k + 1:, k:] -= f[:, None] * A[k, k:][None, :]
        b[k + 1:] -= f * b[k]
    x = np.zeros(n, dtype=np.longdouble)
    for k in reversed(range(n)):
        x[k] = (b[k] - A[k, k + 1:] @ x[k + 1:]) / A[k, k]
    return x


@pytest.mark.parametrize("iters", [1, 3])
def test_kkt_solution_against_dense_elimination(tmp_path, iters):
    T = 20
    prog = cartpole_mpc(T=T, iters=iters, outputs="debug")
    x0 = inputs.cartpole_state(103, 12)
    z, sol, rhs, Af, Bf, huu, D = run(prog, [x0], tmp_path, name=f"dbg{iters}")
    ix, il, iu, n = kkt_index(T)
    assert sol.shape[0] == n
    for i in range(x0.shape[1]):
        A = Af[:, i].reshape(T, NX, NX)
        B = Bf[:, i].reshape(T, NX)
        K = _assemble(T, A, B, huu[:, i])
        r = rhs[:, i].astype(np.longdouble)
        v = sol[:, i].astype(np.longdouble)
        res = np.max(np.abs(K @ v - r)) / np.max(np.abs(r))
        assert res <= 1e-12, (i, res)
        ref = _solve_ld(K, r)
        assert np.max(np.abs(v - ref)) <= 1e-11 * np.max(np.abs(ref)), i
        # pivot signs of the chosen order
        for k in range(T + 1):
            assert np.all(D[ix[k]:ix[k] + NX, i] > 0)
            assert np.all(D[il[k]:il[k] + NX, i] < 0)
            if k < T:
                assert D[iu[k], i] > 0
        # the penalty Hessian is R or R + 2 mu, never anything else
        mu_last = 10.0 * 10.0 ** (iters - 1)
        assert np.all(np.isclose(huu[:, i], R) | np.isclose(huu[:, i], R + 2 * mu_last))


def _cp_invariants(x, cp=CartPole()):
    _, th, xd, thd = x
    mt = cp.mc + cp.mp
    E = 0.5 * mt * xd ** 2 + cp.mp * cp.l * xd * thd * np.cos(th) + 0.5 * cp.mp * cp.l ** 2 * thd ** 2 \
        + cp.mp * cp.grav * cp.l * np.cos(th)
    p = mt * xd + cp.mp * cp.l * thd * np.cos(th)
    return E, p


def test_cartpole_rk4_conserves_energy_and_momentum(tmp_path):
    x = inputs.cartpole_state(5, 64)
    x[1] *= 0.5
    E0, p0 = _cp_invariants(x)
    errs = []
    for dt in (0.04, 0.02):
        x1 = run(cartpole_step(dt), [x, np.zeros((1, 64))], tmp_path, name=f"cp{dt}")[0]
        E1, p1 = _cp_invariants(x1)
        errs.append((np.abs(E1 - E0), np.abs(p1 - p0)))
    rE = np.median(errs[0][0] / errs[1][0])
    rp = np.median(errs[0][1] / errs[1][1])
    assert 20 < rE < 45, rE
    assert 20 < rp < 45, rp


def test_defect_falls_over_iterations_near_upright(tmp_path):
    T = 20
    N = 64
    rng = np.random.default_rng(2)
    x0 = np.stack([rng.uniform(-1, 1, N), rng.uniform(-0.3, 0.3, N), rng.uniform(-1, 1, N),
                   rng.uniform(-1, 1, N)])
    step = cartpole_step(0.02)
    med = []
    for iters in (1, 2, 3):
        z = run(cartpole_mpc(T=T, iters=iters), [x0], tmp_path, name=f"d{iters}")[0]
        X = z[:4 * (T + 1)].reshape(T + 1, 4, N)
        U = z[4 * (T + 1):].reshape(T, N)
        dmax = np.zeros(N)
        for k in range(T):
            f = run(step, [X[k], U[k][None, :]], tmp_path, name="st")[0]
            dmax = np.maximum(dmax, np.max(np.abs(X[k + 1] - f), axis=0))
        med.append(np.median(dmax))
    assert med[1] < 0.1 * med[0] and med[2] < 0.1 * med[1], med


@pytest.mark.slow
def test_inherent_sensitivity_mpc(tmp_path):
    x = inputs.cartpole_state(103, 4096)
    prog = cartpole_mpc()
    y64 = run(prog, [x], tmp_path, 64)[0]
    y80 = run(prog, [x], tmp_path, 80)[0]
    sc = np.sqrt(np.mean(y80 ** 2, axis=1, keepdims=True))
    err = np.abs(y64 - y80) / np.maximum(np.abs(y80), sc)
    assert err.max() <= 1e-11
    assert np.all(np.isfinite(y64))


def test_iterates_converge_over_the_iteration_sweep(tmp_path):
    """M = 1 .. 5: the SQP step between successive fixed-iteration results
    shrinks by at least 5x per added iteration for instances near upright
    (the sweep's M = 1 is the real-time-iteration variant)."""
    T, N = 20, 64
    rng = np.random.default_rng(5)
    x0 = np.stack([rng.uniform(-1, 1, N), rng.uniform(-0.3, 0.3, N), rng.uniform(-1, 1, N),
                   rng.uniform(-1, 1, N)])
    zs = [run(cartpole_mpc(T=T, iters=m), [x0], tmp_path, name=f"s{m}")[0] for m in range(1, 6)]
    steps = [np.median(np.max(np.abs(zs[m + 1] - zs[m]), axis=0)) for m in range(4)]
    assert all(steps[m + 1] < 0.2 * steps[m] for m in range(3)), steps


@pytest.mark.slow
def test_inherent_sensitivity_mpc_five_iterations(tmp_path):
    x = inputs.cartpole_state(103, 1024)
    prog = cartpole_mpc(iters=5)
    y64 = run(prog, [x], tmp_path, 64)[0]
    y80 = run(prog, [x], tmp_path, 80)[0]
    sc = np.sqrt(np.mean(y80 ** 2, axis=1, keepdims=True))
    assert (np.abs(y64 - y80) / np.maximum(np.abs(y80), sc)).max() <= 1e-11
