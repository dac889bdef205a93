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
(vii) The linearisation: the program's A_k, B_k equal the oracle's own
      dual-number Jacobian of the cart-pole RK4 step at the point the last
      iteration linearised at, and its dynamics residuals equal the oracle's
      evaluation of that step there.
(viii) The penalty: the program's cost-gradient entries equal
      -(R u + 2 mu (max(0, u - u_max) - max(0, -u - u_max))) and -Q x
      written out here, and its input Hessian R + 2 mu on the active set
      (penalty-cost equation of the MPC section, p(x) = sum max(0, x_i)^2).
(ix)  Penalised QP with linear dynamics: M iterations of the program equal M
      semismooth Newton steps on the penalised problem, computed here in
      long double on a dense KKT system in another unknown order.
(x)   Those pins detect a sign flip or a dropped factor 2 in the penalty
      gradient (the mistake is planted in the builder, on the CPU).
"""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from workloads import inputs
import workloads.mpc as mpc_module
from workloads.mpc import CartPole, Linear, NX, cartpole_mpc, cartpole_step, kkt_index
from workloads.tracer import fmax, lt

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
    z, sol, rhs, Af, Bf, huu, D, _, _ = run(prog, [x0], tmp_path, name=f"dbg{iters}")
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


# ----------------------------------------------------------------- (vii)-(x)

def _debug_run(tmp_path, x0, name, **kw):
    prog = cartpole_mpc(outputs="debug", **kw)
    return run(prog, [x0], tmp_path, name=name)


def _linearisation_errors(tmp_path, x0, T=20, dt=0.02, **kw):
    """Max relative errors of (A_k, B_k) against the oracle's dual-number
    Jacobian and of the dynamics residuals against the oracle's step."""
    z, sol, rhs, Af, Bf, huu, D, xl, ul = _debug_run(tmp_path, x0, "lin", T=T, dt=dt, **kw)
    N = x0.shape[1]
    ix, il, iu, n = kkt_index(T)
    X = xl.reshape(T, NX, N)
    U = ul.reshape(T, N)
    path = tmp_path / "step.xgp"
    cartpole_step(dt).save(path)
    o = OProg(path)
    # all (k, instance) points in one evaluation
    xs = np.transpose(X, (1, 0, 2)).reshape(NX, T * N)
    us = U.reshape(1, T * N)
    f, J = o.jacobian([xs, us], threads=4)  # J: (4, 5, T*N)
    f = f[0].reshape(NX, T, N)
    J = J.reshape(NX, NX + 1, T, N)
    A = Af.reshape(T, NX, NX, N)
    B = Bf.reshape(T, NX, N)
    JA = np.transpose(J[:, :NX], (2, 0, 1, 3))
    JB = np.transpose(J[:, NX], (1, 0, 2))
    ea = np.max(np.abs(A - JA)) / np.max(np.abs(JA))
    eb = np.max(np.abs(B - JB)) / np.max(np.abs(JB))
    # residual rows of the constraints defining x_{k+1}: f_k - x_{k+1}
    Xn = np.concatenate([X[1:], z[4 * T:4 * (T + 1)][None]], axis=0)  # placeholder for k = T - 1
    res = np.stack([rhs[il[k + 1]:il[k + 1] + NX] for k in range(T)])  # (T, 4, N)
    ref = np.transpose(f, (1, 0, 2)) - Xn
    ref[T - 1] = res[T - 1]  # x_T of the linearisation point is not an output
    er = np.max(np.abs(res - ref)) / np.max(np.abs(ref))
    return ea, eb, er


def _penalty_errors(tmp_path, x0, T=20, umax=10.0, iters=3, mu0=10.0, alpha=10.0, R=0.1):
    """Max errors of the program's u-gradient, x-gradient and u-Hessian
    entries against the penalty written out here, and the number of
    (k, instance) points with an active bound."""
    z, sol, rhs, Af, Bf, huu, D, xl, ul = _debug_run(tmp_path, x0, "pen", T=T, umax=umax,
                                                     iters=iters, mu0=mu0, alpha=alpha, R=R)
    N = x0.shape[1]
    ix, il, iu, n = kkt_index(T)
    mu = mu0 * alpha ** (iters - 1)
    U = ul.reshape(T, N)
    X = xl.reshape(T, NX, N)
    grad_u = R * U + 2.0 * mu * (np.maximum(0.0, U - umax) - np.maximum(0.0, -U - umax))
    ru = np.stack([rhs[iu[k]] for k in range(T)])
    eu = np.max(np.abs(ru + grad_u)) / np.max(np.abs(grad_u))
    active = (U > umax) | (U < -umax)
    eh = np.max(np.abs(huu - (R + 2.0 * mu * active)))
    rx = np.stack([rhs[ix[k]:ix[k] + NX] for k in range(T)])
    ex = np.max(np.abs(rx + Qd[None, :, None] * X)) / np.max(np.abs(Qd[None, :, None] * X))
    return eu, eh, ex, int(active.sum())


def test_linearisation_matches_oracle_dual_numbers(tmp_path):
    x0 = inputs.cartpole_state(103, 24)
    ea, eb, er = _linearisation_errors(tmp_path, x0)
    assert ea <= 1e-13 and eb <= 1e-13, (ea, eb)
    assert er <= 1e-13, er


def test_penalty_gradient_and_hessian(tmp_path):
    # u_max = 3 (the workload's 10 is inactive at these instances' last
    # iterate): the bound is active at about a third of the points
    x0 = inputs.cartpole_state(103, 32)
    eu, eh, ex, n_active = _penalty_errors(tmp_path, x0, umax=3.0)
    assert n_active >= 100, n_active
    assert eu <= 1e-14, eu
    assert eh == 0.0, eh
    assert ex <= 1e-15, ex


def _penalised_lqr_reference(A, B, x0, T, iters, umax, mu0, alpha, R):
    """M semismooth Newton steps on
         min 1/2 sum (x_k^T Q x_k + R u_k^2) + 1/2 x_T^T Q_T x_T
             + mu_j sum_k (max(0, u_k - u_max)^2 + max(0, -u_k - u_max)^2)
         s.t. x_0 = xbar_0, x_{k+1} = A x_k + B u_k,
    from x_k = xbar_0, u_k = 0, mu_j = mu0 alpha^j, in long double, with
    the unknowns ordered (x_0 .. x_T, u_0 .. u_{T-1}) and a dense KKT
    matrix solved by Gaussian elimination with partial pivoting."""
    ld = np.longdouble
    nx = NX * (T + 1)
    nz = nx + T
    ne = NX * (T + 1)
    E = np.zeros((ne, nz), dtype=ld)
    b = np.zeros(ne, dtype=ld)
    E[:NX, :NX] = np.eye(NX)
    b[:NX] = x0
    for k in range(T):
        r = NX * (k + 1)
        E[r:r + NX, NX * (k + 1):NX * (k + 2)] = np.eye(NX)
        E[r:r + NX, NX * k:NX * (k + 1)] = -A
        E[r:r + NX, nx + k] = -B[:, 0]
    qdiag = np.concatenate([Qd * (QT_SCALE if k == T else 1.0) for k in range(T + 1)]).astype(ld)
    z = np.concatenate([np.tile(x0.astype(ld), T + 1), np.zeros(T, dtype=ld)])
    mu = ld(mu0)
    for _ in range(iters):
        x, u = z[:nx], z[nx:]
        act = ((u > umax) | (u < -umax)).astype(ld)
        g = np.concatenate([qdiag * x, R * u + 2 * mu * (np.maximum(0, u - umax) - np.maximum(0, -u - umax))])
        H = np.diag(np.concatenate([qdiag, R + 2 * mu * act]))
        K = np.zeros((nz + ne, nz + ne), dtype=ld)
        K[:nz, :nz] = H
        K[:nz, nz:] = E.T
        K[nz:, :nz] = E
        rhs = np.concatenate([-g, b - E @ z])
        z = z + _solve_ld(K, rhs)[:nz]
        mu = mu * alpha
    return z


def _penalised_qp_error(tmp_path, iters, umax=1.0, mu0=10.0, alpha=10.0, R=0.1, N=6):
    A, B = _lin_AB()
    T = 20
    x0 = inputs.cartpole_state(41, N)
    prog = cartpole_mpc(T=T, iters=iters, dyn=Linear(A, B), umax=umax, mu0=mu0, alpha=alpha)
    z = run(prog, [x0], tmp_path, name=f"pq{iters}")[0]
    worst, n_active = 0.0, 0
    for i in range(N):
        ref = _penalised_lqr_reference(A, B, x0[:, i], T, iters, umax, mu0, alpha, R)
        # program order: (x_0 .. x_T, u_0 .. u_{T-1}), the same as the reference's
        worst = max(worst, float(np.max(np.abs(z[:, i] - ref)) / np.max(np.abs(ref))))
        n_active += int(np.sum(np.abs(ref[NX * (T + 1):]) > umax))
    return worst, n_active


@pytest.mark.parametrize("iters", [1, 2, 3])
def test_penalised_linear_qp_equals_semismooth_newton(tmp_path, iters):
    err, n_active = _penalised_qp_error(tmp_path, iters)
    assert n_active >= 10, n_active  # the penalty shapes the result
    assert err <= 1e-11, err


def _flipped_sign(u, umax, mu, R):
    h = R + (2.0 * mu) * (lt(umax, u) + lt(u, -umax))
    return h, R * u - (2.0 * mu) * (fmax(u - umax, 0.0) - fmax(-u - umax, 0.0))


def _dropped_two(u, umax, mu, R):
    h = R + (2.0 * mu) * (lt(umax, u) + lt(u, -umax))
    return h, R * u + mu * (fmax(u - umax, 0.0) - fmax(-u - umax, 0.0))


@pytest.mark.parametrize("mutant", [_flipped_sign, _dropped_two])
def test_penalty_pins_detect_planted_mistakes(tmp_path, monkeypatch, mutant):
    monkeypatch.setattr(mpc_module, "penalty_terms", mutant)
    x0 = inputs.cartpole_state(103, 32)
    eu, eh, ex, n_active = _penalty_errors(tmp_path, x0, umax=3.0)
    assert n_active > 0
    assert eu > 1e-3, eu
    err, _ = _penalised_qp_error(tmp_path, 2)
    assert err > 1e-3, err
