"""Planar n-link serial pendulum, one RK4 step, as one straight-line program.

Recipe (a reading; the workload description fixes only "unit masses and
lengths, mass matrix + Coriolis + gravity, forward dynamics by unrolled
Cholesky, one RK4 step"):

* point masses m_i at the tips of massless links of length l_i, g = 9.81;
* joint (relative) angles q, q_1 measured from the downward vertical,
  absolute angles phi_i = q_1 + ... + q_i, tip positions
  p_i = sum_{j<=i} l_j (sin phi_j, -cos phi_j);
* M(q) = sum_i m_i J_i^T J_i with J_i = dp_i/dq (symbolic Jacobian);
* Coriolis/centrifugal term (C qd)_k = sum_{ij} Gamma_kij qd_i qd_j with the
  Christoffel symbols Gamma_kij = (dM_kj/dq_i + dM_ki/dq_j - dM_ij/dq_k)/2;
* gravity G = dV/dq with V = g sum_i m_i p_{i,y};
* qdd = M^{-1}(-C qd - G) by an unrolled Cholesky factorisation M = L L^T
  followed by forward and back substitution;
* state s = (q, qd) as one input argument; one classical RK4 step.
"""

from __future__ import annotations

from .tracer import Graph, Sym, sin, cos, sqrt

G_ACC = 9.81


def _accel(g: Graph, q, qd, m, l, grav, debug=None):
    n = len(q)
    phi = []
    acc = None
    for i in range(n):
        acc = q[i] if acc is None else acc + q[i]
        phi.append(acc)
    sp = [sin(p) for p in phi]
    cp = [cos(p) for p in phi]
    px, py = [], []
    ax = ay = None
    for i in range(n):
        tx = l[i] * sp[i]
        ty = -(l[i] * cp[i])
        ax = tx if ax is None else ax + tx
        ay = ty if ay is None else ay + ty
        px.append(ax)
        py.append(ay)
    Jx = g.jacobian(px, q)
    Jy = g.jacobian(py, q)
    zero = g.const(0.0)
    J = lambda Jm, i, k: Jm[i][k] if Jm[i][k] is not None else zero  # noqa: E731
    # mass matrix, lower triangle (symmetric: M[k][l] is M[l][k])
    M = [[None] * n for _ in range(n)]
    tri = []
    for k in range(n):
        for c in range(k + 1):
            s = None
            for i in range(n):
                t = m[i] * (J(Jx, i, k) * J(Jx, i, c) + J(Jy, i, k) * J(Jy, i, c))
                s = t if s is None else s + t
            M[k][c] = M[c][k] = s
            tri.append((k, c))
    dMl = g.jacobian([M[k][c] for (k, c) in tri], q)
    dM = {}
    for r, (k, c) in enumerate(tri):
        for i in range(n):
            d = dMl[r][i] if dMl[r][i] is not None else zero
            dM[(k, c, i)] = dM[(c, k, i)] = d
    # Coriolis/centrifugal: (C qd)_k = sum_ij Gamma_kij qd_i qd_j
    cor = []
    for k in range(n):
        s = None
        for i in range(n):
            for j in range(n):
                gam = 0.5 * (dM[(k, j, i)] + dM[(k, i, j)] - dM[(i, j, k)])
                t = gam * qd[i] * qd[j]
                s = t if s is None else s + t
        cor.append(s)
    V = None
    for i in range(n):
        t = (grav * m[i]) * py[i]
        V = t if V is None else V + t
    Gv = g.jacobian([V], q)[0]
    rhs = [-(cor[k]) - (Gv[k] if Gv[k] is not None else zero) for k in range(n)]
    # unrolled Cholesky M = L L^T
    L = [[None] * n for _ in range(n)]
    for j in range(n):
        s = M[j][j]
        for k in range(j):
            s = s - L[j][k] * L[j][k]
        L[j][j] = sqrt(s)
        for i in range(j + 1, n):
            s = M[i][j]
            for k in range(j):
                s = s - L[i][k] * L[j][k]
            L[i][j] = s / L[j][j]
    y = [None] * n
    for i in range(n):
        s = rhs[i]
        for k in range(i):
            s = s - L[i][k] * y[k]
        y[i] = s / L[i][i]
    qdd = [None] * n
    for i in reversed(range(n)):
        s = y[i]
        for k in range(i + 1, n):
            s = s - L[k][i] * qdd[k]
        qdd[i] = s / L[i][i]
    if debug is not None:
        debug["M"] = [M[k][c] for (k, c) in tri]
        debug["L"] = [L[k][c] for (k, c) in tri]
        debug["rhs"] = rhs
    return qdd


def pendulum(n: int = 7, dt: float = 1e-3, outputs: str = "state",
             masses=None, lengths=None, grav: float = G_ACC,
             dtype: str = "f64", reuse_slots: bool = True):
    """Build the n-link pendulum program.

    outputs:
      "state" -- s' after one RK4 step (2n values);
      "accel" -- qdd at s (n values);
      "debug" -- [qdd], [M lower triangle row-major], [L lower triangle]
    """
    m = list(masses) if masses is not None else [1.0] * n
    l = list(lengths) if lengths is not None else [1.0] * n
    g = Graph(f"pend{n}_{outputs}", dtype)
    s = g.input(2 * n)
    q, qd = s[:n], s[n:]
    if outputs in ("accel", "debug"):
        dbg: dict = {}
        qdd = _accel(g, q, qd, m, l, grav, dbg)
        if outputs == "accel":
            return g.program([qdd], reuse_slots)
        return g.program([qdd, dbg["M"], dbg["L"]], reuse_slots)
    if outputs != "state":
        raise ValueError(outputs)

    def f(qq, vv):
        return list(vv), _accel(g, qq, vv, m, l, grav)

    h2, h6 = dt / 2.0, dt / 6.0
    k1q, k1v = f(q, qd)
    k2q, k2v = f([q[i] + h2 * k1q[i] for i in range(n)], [qd[i] + h2 * k1v[i] for i in range(n)])
    k3q, k3v = f([q[i] + h2 * k2q[i] for i in range(n)], [qd[i] + h2 * k2v[i] for i in range(n)])
    k4q, k4v = f([q[i] + dt * k3q[i] for i in range(n)], [qd[i] + dt * k3v[i] for i in range(n)])
    qn = [q[i] + h6 * (k1q[i] + 2.0 * k2q[i] + 2.0 * k3q[i] + k4q[i]) for i in range(n)]
    vn = [qd[i] + h6 * (k1v[i] + 2.0 * k2v[i] + 2.0 * k3v[i] + k4v[i]) for i in range(n)]
    return g.program([qn + vn], reuse_slots)


def pendulum_gradient_seed_note() -> str:
    """The adjoint workload: L = ||s'||^2, so dL/ds = J^T (2 s')."""
    return "seed ybar = 2 s'"


__all__ = ["pendulum", "G_ACC", "Sym"]
