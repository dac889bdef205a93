"""Physics pins of the pendulum program as evaluated by the oracle.

None of these compare the oracle with itself: each checks the program's
result against mechanics that fix it independently --
(i) one link reduces to thetadd = -(g/l) sin theta;
(ii) two links equal the textbook double-pendulum equations (absolute
     angles, arbitrary masses and lengths);
(iii) seven links equal the compact absolute-angle Lagrangian form
     M_jk = l_j l_k mu_max(j,k) cos(phi_j - phi_k),
     c_j = sum_k l_j l_k mu_max(j,k) sin(phi_j - phi_k) phidot_k^2,
     G_j = g l_j mu_j sin phi_j (mu_k = sum_{i>=k} m_i), solved by numpy
     in long double and mapped to joint angles by phi = T q;
(iv) the mass matrix is symmetric positive definite and L L^T = M;
(v) q = 0, qdot = 0 is an exact fixed point;
(vi) the RK4 step's energy error shrinks ~32x when dt halves (local order 5);
plus the inherent sensitivity of the 7-link step (long double vs double).
"""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from workloads import inputs
from workloads.pendulum import pendulum

G = 9.81


def run(prog, x, tmp_path, scalar=64, name="p"):
    path = tmp_path / f"{name}.xgp"
    prog.save(path)
    return OProg(path).evaluate(x, scalar)


def compact_accel(q, qd, m, l, g=G):
    """q, qd: (n,) long double.  Absolute-angle Lagrangian form."""
    n = len(q)
    ld = np.longdouble
    T = np.tril(np.ones((n, n), dtype=ld))
    phi = T @ q
    phid = T @ qd
    mu = np.array([sum(m[i:]) for i in range(n)], dtype=ld)
    Mp = np.empty((n, n), dtype=ld)
    c = np.zeros(n, dtype=ld)
    for j in range(n):
        for k in range(n):
            w = ld(l[j]) * ld(l[k]) * mu[max(j, k)]
            Mp[j, k] = w * np.cos(phi[j] - phi[k])
            c[j] += w * np.sin(phi[j] - phi[k]) * phid[k] ** 2
    Gp = np.array([ld(g) * ld(l[j]) * mu[j] * np.sin(phi[j]) for j in range(n)], dtype=ld)
    phidd = _solve_ld(Mp, -(c + Gp))
    qdd = np.empty(n, dtype=ld)
    qdd[0] = phidd[0]
    qdd[1:] = phidd[1:] - phidd[:-1]  # T^{-1}
    return qdd, Mp, T


def _solve_ld(A, b):
    """Gaussian elimination with partial pivoting in long double."""
    A = A.astype(np.longdouble).copy()
    b = b.astype(np.longdouble).copy()
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


def test_single_link_reduces_to_simple_pendulum(tmp_path):
    rng = np.random.default_rng(3)
    s = np.stack([rng.uniform(-np.pi, np.pi, 64), rng.normal(size=64)])
    for length in (1.0, 0.7):
        qdd = run(pendulum(1, outputs="accel", lengths=[length]), [s], tmp_path)[0][0]
        ref = -(G / length) * np.sin(s[0])
        assert np.max(np.abs(qdd - ref)) <= 4e-15 * G / length


def test_two_links_match_textbook_double_pendulum(tmp_path):
    m1, m2, L1, L2 = 1.3, 0.7, 0.9, 1.4
    rng = np.random.default_rng(4)
    n = 64
    q = rng.uniform(-np.pi, np.pi, (2, n))
    qd = rng.normal(size=(2, n))
    out = run(pendulum(2, outputs="accel", masses=[m1, m2], lengths=[L1, L2]),
              [np.concatenate([q, qd])], tmp_path)[0]
    t1, t2 = q[0], q[0] + q[1]
    w1, w2 = qd[0], qd[0] + qd[1]
    den = 2 * m1 + m2 - m2 * np.cos(2 * t1 - 2 * t2)
    a1 = (-G * (2 * m1 + m2) * np.sin(t1) - m2 * G * np.sin(t1 - 2 * t2)
          - 2 * np.sin(t1 - t2) * m2 * (w2 ** 2 * L2 + w1 ** 2 * L1 * np.cos(t1 - t2))) / (L1 * den)
    a2 = (2 * np.sin(t1 - t2) * (w1 ** 2 * L1 * (m1 + m2) + G * (m1 + m2) * np.cos(t1)
                                 + w2 ** 2 * L2 * m2 * np.cos(t1 - t2))) / (L2 * den)
    ref = np.stack([a1, a2 - a1])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(out - ref)) <= 1e-12 * scale


def test_seven_links_match_compact_absolute_angle_form(tmp_path):
    n, N = 7, 48
    m = [1.0, 0.8, 1.2, 1.0, 0.9, 1.1, 1.0]
    l = [1.0, 0.9, 1.1, 1.0, 1.2, 0.8, 1.0]
    s = inputs.pendulum_state(21, n, N)
    res = run(pendulum(n, outputs="debug", masses=m, lengths=l), [s], tmp_path)
    qdd, Mtri, Ltri = res
    for i in range(N):
        ref, Mp, T = compact_accel(s[:n, i].astype(np.longdouble), s[n:, i].astype(np.longdouble), m, l)
        ref = ref.astype(np.float64)
        assert np.max(np.abs(qdd[:, i] - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref))), i
        # (iv) mass matrix = T^T M_phi T, symmetric positive definite, L L^T = M
        Mq = (T.T @ Mp @ T).astype(np.float64)
        Mfull = np.zeros((n, n))
        Lfull = np.zeros((n, n))
        r = 0
        for k in range(n):
            for c in range(k + 1):
                Mfull[k, c] = Mfull[c, k] = Mtri[r, i]
                Lfull[k, c] = Ltri[r, i]
                r += 1
        assert np.max(np.abs(Mfull - Mq)) <= 1e-13 * np.max(np.abs(Mq))
        assert np.all(np.linalg.eigvalsh(Mfull) > 0)
        assert np.all(np.diag(Lfull) > 0)
        assert np.max(np.abs(Lfull @ Lfull.T - Mfull)) <= 1e-14 * np.max(np.abs(Mfull)) * n


def test_rest_is_exact_fixed_point(tmp_path):
    y = run(pendulum(7), [np.zeros((14, 5))], tmp_path)[0]
    assert np.array_equal(y, np.zeros((14, 5)))


def _energy(s, m, l, n):
    E = []
    for i in range(s.shape[1]):
        q = s[:n, i].astype(np.longdouble)
        qd = s[n:, i].astype(np.longdouble)
        _, Mp, T = compact_accel(q, qd, m, l)
        phi = T @ q
        phid = T @ qd
        mu = [sum(m[k:]) for k in range(n)]
        V = -G * sum(l[j] * mu[j] * np.cos(phi[j]) for j in range(n))
        E.append(0.5 * phid @ Mp @ phid + V)
    return np.array(E, dtype=np.float64)


def test_rk4_energy_error_is_fifth_order(tmp_path):
    n, N = 7, 16
    m = [1.0] * n
    l = [1.0] * n
    rng = np.random.default_rng(8)
    s = np.concatenate([rng.uniform(-0.6, 0.6, (n, N)), 0.3 * rng.normal(size=(n, N))])
    E0 = _energy(s, m, l, n)
    errs = []
    for dt in (0.02, 0.01):
        s1 = run(pendulum(n, dt=dt), [s], tmp_path, name=f"e{dt}")[0]
        errs.append(np.abs(_energy(s1, m, l, n) - E0))
    ratio = np.median(errs[0] / errs[1])
    assert 20.0 < ratio < 45.0, ratio


def test_inherent_sensitivity_pendulum(tmp_path):
    s = inputs.pendulum_state(102, 7, 512)
    prog = pendulum(7)
    y64 = run(prog, [s], tmp_path, 64)[0]
    y80 = run(prog, [s], tmp_path, 80)[0]
    sc = np.sqrt(np.mean(y80 ** 2, axis=1, keepdims=True))
    err = np.abs(y64 - y80) / np.maximum(np.abs(y80), sc)
    assert err.max() <= 1e-13


@pytest.mark.slow
def test_fp32_inherent_error_is_small(tmp_path):
    s = inputs.pendulum_state(102, 7, 512)
    s32 = s.astype(np.float32).astype(np.float64)
    prog = pendulum(7)
    y32 = run(prog, [s32], tmp_path, 32)[0]
    y64 = run(prog, [s32], tmp_path, 64)[0]
    sc = np.sqrt(np.mean(y64 ** 2, axis=1, keepdims=True))
    err = np.abs(y32 - y64) / np.maximum(np.abs(y64), sc)
    assert err.max() <= 2.5e-6
