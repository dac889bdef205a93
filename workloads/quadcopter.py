"""Closed-loop step of a planar quadcopter under an infinite-horizon LQR
controller (the paper's quadcopter application): z_{k+1} = f(z_k, theta).

Readings where the paper is silent:

* model: the textbook planar quadrotor, state z = (x, y, phi, xdot, ydot,
  phidot), inputs the two rotor thrusts (u1, u2):
      xddot = -(u1 + u2) sin(phi) / m,  yddot = (u1 + u2) cos(phi) / m - g,
      phiddot = r (u1 - u2) / I;
* integrator: semi-implicit Euler with dt = 0.01 (velocities first, then
  positions with the new velocities);
* controller: LQR about hover at the origin (phi = 0, u1 = u2 = m g / 2)
  for the discrete linearisation of that step, whose A and B are formed
  symbolically from the parameters by dual numbers;
* the discrete algebraic Riccati equation is solved by the structured
  doubling algorithm with a fixed number of iterations (12, within the
  10-15 the paper found suitable), written in the form that needs only
  inverses of symmetric positive definite matrices (unrolled Cholesky):
      M_k = H_k^{-1} + G_k,
      A_{k+1} = A_k H_k^{-1} M_k^{-1} A_k,
      G_{k+1} = G_k + A_k H_k^{-1} M_k^{-1} G_k A_k^T,
      H_{k+1} = H_k + A_k^T M_k^{-1} A_k,
  from A_0 = A, G_0 = B R^{-1} B^T, H_0 = Q; H_k tends to the Riccati
  solution S (this is the standard doubling recursion with
  (I + G H)^{-1} = H^{-1} (H^{-1} + G)^{-1}, valid since H_k >= Q > 0);
* gain K = (R + B^T S B)^{-1} B^T S A; thrusts u = u_hover - K z, each
  clamped to [0, u_max] (branch-free through min/max);
* parameters theta (the second input, 12 values): m, I, r, u_max,
  Q diagonal (6), R diagonal (2); g = 9.81.
"""

from __future__ import annotations

import numpy as np

from .tracer import Dual, Graph, cos, fmax, fmin, sin

NZ, NU, NTH = 6, 2, 12
GRAV = 9.81


def quad_step(z, u, m, inertia, arm, dt):
    """Semi-implicit Euler step of the planar quadrotor (works on Syms or Duals)."""
    x, y, phi, xd, yd, phid = z
    T = u[0] + u[1]
    s, c = sin(phi), cos(phi)
    xdd = -(T * s) / m
    ydd = (T * c) / m - GRAV
    phidd = ((u[0] - u[1]) * arm) / inertia
    xd1 = xd + dt * xdd
    yd1 = yd + dt * ydd
    phid1 = phid + dt * phidd
    return [x + dt * xd1, y + dt * yd1, phi + dt * phid1, xd1, yd1, phid1]


def _mat(rows):
    return [list(r) for r in rows]


def _mm(A, B, zero):
    n, k, m = len(A), len(B), len(B[0])
    out = []
    for i in range(n):
        row = []
        for j in range(m):
            s = None
            for t in range(k):
                a, b = A[i][t], B[t][j]
                if _is_zero(a) or _is_zero(b):
                    continue
                p = a * b
                s = p if s is None else s + p
            row.append(zero if s is None else s)
        out.append(row)
    return out


def _is_zero(v):
    return v is None or (hasattr(v, "is_zero") and v.is_zero())


def _T(A):
    return [list(r) for r in zip(*A)]


def _sym_add(A, B):
    """A + B for symmetric A, B: upper triangle computed once, mirrored."""
    n = len(A)
    out = [[None] * n for _ in range(n)]
    for i in range(n):
        for j in range(i, n):
            out[i][j] = out[j][i] = A[i][j] + B[i][j]
    return out


def _chol(S):
    n = len(S)
    L = [[None] * n for _ in range(n)]
    for j in range(n):
        d = S[j][j]
        for k in range(j):
            d = d - L[j][k] * L[j][k]
        from .tracer import sqrt
        L[j][j] = sqrt(d)
        for i in range(j + 1, n):
            s = S[i][j]
            for k in range(j):
                s = s - L[i][k] * L[j][k]
            L[i][j] = s / L[j][j]
    return L


def _chol_solve(L, Bm):
    """Solve (L L^T) X = Bm column by column."""
    n, m = len(L), len(Bm[0])
    X = [[None] * m for _ in range(n)]
    for c in range(m):
        y = []
        for i in range(n):
            s = Bm[i][c]
            for k in range(i):
                s = s - L[i][k] * y[k]
            y.append(s / L[i][i])
        x = [None] * n
        for i in reversed(range(n)):
            s = y[i]
            for k in range(i + 1, n):
                s = s - L[k][i] * x[k]
            x[i] = s / L[i][i]
        for i in range(n):
            X[i][c] = x[i]
    return X


def _spd_inverse(S, g):
    n = len(S)
    L = _chol(S)
    E = [[g.const(1.0 if i == j else 0.0) for j in range(n)] for i in range(n)]
    X = _chol_solve(L, E)
    # symmetrise exactly: keep the upper triangle
    for i in range(n):
        for j in range(i):
            X[i][j] = X[j][i]
    return X


def linearisation(g, m, inertia, arm, dt):
    """A = d z'/d z, B = d z'/d u of the step at hover, as Syms of the parameters."""
    zero = g.const(0.0)
    uh = (m * GRAV) * 0.5
    zs = Dual.seed([zero] * NZ + [uh, uh])
    out = quad_step(zs[:NZ], zs[NZ:], m, inertia, arm, dt)
    A = [[o.d[j] if o.d[j] is not None else zero for j in range(NZ)] for o in out]
    B = [[o.d[NZ + j] if o.d[NZ + j] is not None else zero for j in range(NU)] for o in out]
    return A, B


def quad_closed_loop(sda_iters: int = 12, dt: float = 0.01, dtype: str = "f64",
                     outputs: str = "state", reuse_slots: bool = True):
    """z_{k+1} = f(z_k, theta).  outputs: "state" -> [z'];
    "debug" -> [z'], [u (clamped thrusts)], [K (row-major 2x6)], [S (6x6)]."""
    g = Graph(f"quad_lqr_sda{sda_iters}", dtype)
    z = g.input(NZ)
    th = g.input(NTH)
    m, inertia, arm, umax = th[0], th[1], th[2], th[3]
    Qd, Rd = th[4:10], th[10:12]
    zero = g.const(0.0)
    A, B = linearisation(g, m, inertia, arm, dt)
    # G0 = B R^{-1} B^T (R diagonal)
    Rinv = [1.0 / Rd[0], 1.0 / Rd[1]]
    G = [[None] * NZ for _ in range(NZ)]
    for i in range(NZ):
        for j in range(i, NZ):
            s = None
            for k in range(NU):
                if _is_zero(B[i][k]) or _is_zero(B[j][k]):
                    continue
                p = (B[i][k] * Rinv[k]) * B[j][k]
                s = p if s is None else s + p
            G[i][j] = G[j][i] = zero if s is None else s
    H = [[Qd[i] if i == j else zero for j in range(NZ)] for i in range(NZ)]
    Ak = A
    for _ in range(sda_iters):
        Hi = _spd_inverse(H, g)
        M = _sym_add(Hi, G)
        LM = _chol(M)
        Z = _chol_solve(LM, Ak)          # M^{-1} A_k
        Y = _chol_solve(LM, G)           # M^{-1} G_k
        AtZ = _mm(_T(Ak), Z, zero)
        Hn = [[None] * NZ for _ in range(NZ)]
        for i in range(NZ):
            for j in range(i, NZ):
                Hn[i][j] = Hn[j][i] = H[i][j] + AtZ[i][j]
        AHi = _mm(Ak, Hi, zero)
        An = _mm(AHi, Z, zero)
        W = _mm(_mm(AHi, Y, zero), _T(Ak), zero)
        Gn = [[None] * NZ for _ in range(NZ)]
        for i in range(NZ):
            for j in range(i, NZ):
                Gn[i][j] = Gn[j][i] = G[i][j] + W[i][j]
        Ak, G, H = An, Gn, Hn
    S = H
    BtS = _mm(_T(B), S, zero)                       # 2 x 6
    Rb = _mm(BtS, B, zero)                           # 2 x 2
    r00, r01, r11 = Rd[0] + Rb[0][0], Rb[0][1], Rd[1] + Rb[1][1]
    det = r00 * r11 - r01 * r01
    Rbi = [[r11 / det, -(r01 / det)], [-(r01 / det), r00 / det]]
    K = _mm(Rbi, _mm(BtS, A, zero), zero)           # 2 x 6
    uh = (m * GRAV) * 0.5
    u = []
    for k in range(NU):
        v = uh
        for j in range(NZ):
            v = v - K[k][j] * z[j]
        u.append(fmin(fmax(v, zero), umax))
    z1 = quad_step(z, u, m, inertia, arm, dt)
    if outputs == "state":
        return g.program([z1], reuse_slots=reuse_slots)
    if outputs == "debug":
        return g.program([z1, u, [K[i][j] for i in range(NU) for j in range(NZ)],
                          [S[i][j] for i in range(NZ) for j in range(NZ)]], reuse_slots=reuse_slots)
    raise ValueError(outputs)


def quad_params(seed: int, n: int) -> np.ndarray:
    """Seeded parameter draws (12, n): m ~ U(0.8, 1.2) kg, I ~ U(0.008, 0.012)
    kg m^2, r ~ U(0.1, 0.2) m, u_max ~ U(0.75, 1.5) m g (per rotor; hover
    needs m g / 2), Q = diag(U(1,10), U(1,10), U(1,10), U(0.1,1) x3),
    R = diag(U(0.1, 1) x2)."""
    rng = np.random.default_rng(seed)
    m = rng.uniform(0.8, 1.2, n)
    inertia = rng.uniform(0.008, 0.012, n)
    arm = rng.uniform(0.1, 0.2, n)
    umax = rng.uniform(0.75, 1.5, n) * m * GRAV
    Q = np.concatenate([rng.uniform(1, 10, (3, n)), rng.uniform(0.1, 1, (3, n))])
    R = rng.uniform(0.1, 1, (2, n))
    return np.ascontiguousarray(np.concatenate([m[None], inertia[None], arm[None], umax[None], Q, R]))


def quad_initial(seed: int, n: int) -> np.ndarray:
    """Initial states for the region-of-attraction rollouts: zero position and
    attitude, linear momenta ~ U(-3, 3) m/s and angular rate ~ U(-6, 6) rad/s."""
    rng = np.random.default_rng(seed)
    z = np.zeros((NZ, n))
    z[3] = rng.uniform(-3, 3, n)
    z[4] = rng.uniform(-3, 3, n)
    z[5] = rng.uniform(-6, 6, n)
    return z
