"""Closed-form MPC: a fixed number of penalty-SQP iterations, each solving
its KKT system by a fixed-pattern LDL^T factorisation without pivoting.

This follows the paper's application section on MPC parallelisation: the
OCP of its Eq. (1) is transcribed into the NLP (z, G^eq, G^ineq, J); one
solver iteration h is an SQP step whose QP (Eq. for the SQP subproblem)
has its inequality constraints moved into the cost as mu * p(.) with the
quadratic penalty p(x) = sum max(0, x_i)^2 (Eq. for the penalty cost);
the equality-constrained QP is solved through LDL^T of its KKT matrix; and
the approximate solution is H(z_0) = h^M(z_0) with a strictly fixed number
of operations.  The penalty grows as mu_{k+1} = alpha mu_k.

Readings where the paper is silent:

* system: cart-pole, state (x, theta, xdot, thetadot), theta = 0 upright,
  point-mass pole, m_c = 1.0, m_p = 0.1, l = 0.5, g = 9.81, input F;
  RK4 with dt = 0.02, horizon T = 20 (dt = 0.05 lets the full-step
  iterates overshoot to |theta| ~ 12 rad, where long-double and double
  evaluations differ by 1e-10; at 0.02 they agree to 6e-13);
* cost 1/2 sum_{k<T} (x_k^T Q x_k + R u_k^2) + 1/2 x_T^T Q_T x_T with
  Q = diag(1, 1, 0.1, 0.1), Q_T = 10 Q, R = 0.1;
* inequality |u_k| <= u_max = 10 as g = (u - u_max, -u - u_max) <= 0;
* mu = 10, 100, 1000 (alpha = 10) over M = 3 iterations;
* Gauss-Newton Hessian (the dynamics' second derivatives are dropped);
  the penalty's Hessian is 2 mu on the currently active set;
* full step (alpha_step = 1; the paper's line search is the branching that
  the closed form removes);
* initial guess x_k = xbar_0 for all k, u_k = 0;
* KKT unknown order (x_0, lam_0, u_0, x_1, lam_1, u_1, ..., x_T, lam_T),
  where lam_k is the multiplier of the constraint that defines x_k.  With
  this order every x/u pivot is the untouched diagonal of Q or R + penalty
  (> 0) and every lam pivot is negative definite, so LDL^T needs no
  pivoting.
"""

from __future__ import annotations

from .tracer import Dual, Graph, sin, cos, fmax, lt

NX, NU = 4, 1


class CartPole:
    def __init__(self, mc=1.0, mp=0.1, l=0.5, grav=9.81):
        self.mc, self.mp, self.l, self.grav = mc, mp, l, grav

    def f(self, x, u):
        """Continuous-time dynamics xdot = f(x, u)."""
        _, th, xd, thd = x
        F = u[0]
        s, c = sin(th), cos(th)
        mc, mp, l, grav = self.mc, self.mp, self.l, self.grav
        den = mc + mp * (s * s)
        xdd = (F + (mp * s) * ((l * thd) * thd - grav * c)) / den
        thdd = (((mc + mp) * grav) * s - F * c - (((mp * l) * thd) * thd) * (s * c)) / (l * den)
        return [xd, thd, xdd, thdd]


def penalty_terms(u, umax, mu, R):
    """Hessian entry and gradient of 1/2 R u^2 + mu p(g(u)) for one input,
    with g(u) = (u - u_max, -u - u_max) and the quadratic penalty
    p(x) = sum max(0, x_i)^2 (penalty-cost equation of the MPC section):
    grad = R u + 2 mu (max(0, u - u_max) - max(0, -u - u_max)), and the
    Gauss-Newton Hessian R + 2 mu on the active set (branch-free through
    FMAX and LT)."""
    hi = u - umax
    lo = -u - umax
    act = lt(umax, u) + lt(u, -umax)
    h = R + (2.0 * mu) * act
    grad = R * u + (2.0 * mu) * (fmax(hi, 0.0) - fmax(lo, 0.0))
    return h, grad


def rk4(dyn, x, u, dt):
    h2, h6 = dt / 2.0, dt / 6.0
    k1 = dyn.f(x, u)
    k2 = dyn.f([x[i] + h2 * k1[i] for i in range(NX)], u)
    k3 = dyn.f([x[i] + h2 * k2[i] for i in range(NX)], u)
    k4 = dyn.f([x[i] + dt * k3[i] for i in range(NX)], u)
    return [x[i] + h6 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]) for i in range(NX)]


class Linear:
    """Discrete-time linear dynamics x+ = A x + B u (for the LQR pin)."""

    def __init__(self, A, B):
        self.A = [[float(v) for v in r] for r in A]
        self.B = [[float(v) for v in r] for r in B]

    def step(self, x, u):
        out = []
        for i in range(NX):
            s = None
            for j in range(NX):
                if self.A[i][j] != 0.0:
                    t = self.A[i][j] * x[j]
                    s = t if s is None else s + t
            for j in range(NU):
                if self.B[i][j] != 0.0:
                    t = self.B[i][j] * u[j]
                    s = t if s is None else s + t
            out.append(s if s is not None else 0.0)
        return out


def _ldl_solve(g: Graph, n: int, K: dict, rhs: list):
    """Fixed-pattern LDL^T solve of K v = rhs (K symmetric, lower part in
    `K[(i, j)]`, i >= j, structural zeros absent).  The fill pattern is
    computed once here; only structural non-zeros become operations."""
    # symbolic factorisation: column patterns of L
    cols = [set() for _ in range(n)]
    rows = [set() for _ in range(n)]  # rows[i] = {k < i : L[i,k] != 0}
    for (i, j) in K:
        if i > j:
            cols[j].add(i)
    for j in range(n):
        for k in sorted(rows[j]):
            for i in cols[k]:
                if i > j:
                    cols[j].add(i)
        for i in cols[j]:
            rows[i].add(j)
    L: dict = {}
    D = [None] * n
    E: dict = {}  # E[(j, k)] = L[j,k] * D[k]
    for j in range(n):
        rj = sorted(rows[j])
        for k in rj:
            E[(j, k)] = L[(j, k)] * D[k]
        s = K.get((j, j))
        for k in rj:
            t = L[(j, k)] * E[(j, k)]
            s = -t if s is None else s - t
        if s is None:
            raise ValueError(f"LDL: structurally zero pivot {j}")
        D[j] = s
        for i in sorted(cols[j]):
            s = K.get((i, j))
            for k in rj:
                if (i, k) in L:
                    t = L[(i, k)] * E[(j, k)]
                    s = -t if s is None else s - t
            if s is None:
                s = g.const(0.0)
            L[(i, j)] = s / D[j]
    # forward solve L y = rhs (unit lower), diagonal, back solve L^T v = w
    y = list(rhs)
    for i in range(n):
        for k in sorted(rows[i]):
            y[i] = y[i] - L[(i, k)] * y[k]
    w = [y[i] / D[i] for i in range(n)]
    v = list(w)
    for i in reversed(range(n)):
        for r in sorted(cols[i]):
            v[i] = v[i] - L[(r, i)] * v[r]
    return v, D


def cartpole_mpc(T: int = 20, iters: int = 3, dt: float = 0.02, umax: float = 10.0,
                 Q=(1.0, 1.0, 0.1, 0.1), QT_scale: float = 10.0, R: float = 0.1,
                 mu0: float = 10.0, alpha: float = 10.0, dyn=None,
                 penalty: bool = True, outputs: str = "z", dtype: str = "f64",
                 reuse_slots: bool = True, precision: str = "f64"):
    """Build the closed-form MPC program H(xbar_0) = h^M(z_0).

    Input: xbar_0 (4).  outputs:
      "z"     -- (x_0..x_T, u_0..u_{T-1}) as one argument of 4(T+1)+T values;
      "debug" -- [z], [KKT solution in unknown order], [rhs], [A_k], [B_k],
                 [H_uu], [D pivots], [x_k, k < T], [u_k] of the LAST iteration
                 (the last two: the point the iteration linearised at).
    `dyn` is a CartPole (continuous, integrated with RK4) or Linear
    (discrete) model.  precision="mixed" computes the dynamics, their
    Jacobians and the cost/penalty terms in binary32 and keeps the KKT
    assembly, the LDL^T factorisation, its pivots, the solves and the
    iterate update in binary64.
    """
    if precision not in ("f64", "mixed"):
        raise ValueError(precision)
    dyn = dyn if dyn is not None else CartPole()
    g = Graph(f"cartpole_mpc_T{T}_M{iters}" + ("_mixed" if precision == "mixed" else ""), dtype)
    low = "f32" if precision == "mixed" else None
    xbar = g.input(NX)
    Qd = [float(v) for v in Q]
    QTd = [QT_scale * v for v in Qd]
    xs = [list(xbar) for _ in range(T + 1)]
    us = [[g.const(0.0)] for _ in range(T)]
    # unknown index map
    ix, il, iu = {}, {}, {}
    n = 0
    for k in range(T + 1):
        ix[k] = n
        n += NX
        il[k] = n
        n += NX
        if k < T:
            iu[k] = n
            n += NU
    dbg = None
    mu = mu0
    for it in range(iters):
        x_lin, u_lin = xs, us  # this iteration's linearisation point
        fk, Ak, Bk = [], [], []
        for k in range(T):
            zd = Dual.seed(xs[k] + us[k])
            with g.precision(low):
                if isinstance(dyn, Linear):
                    fd = dyn.step(zd[:NX], zd[NX:])
                else:
                    fd = rk4(dyn, zd[:NX], zd[NX:], dt)
            fd = [v if isinstance(v, Dual) else Dual(g.lift(v), [None] * (NX + NU)) for v in fd]
            f = [g.lift(v.v) for v in fd]
            fk.append(f)
            Ak.append([[fd[i].d[j] for j in range(NX)] for i in range(NX)])
            Bk.append([[fd[i].d[NX + j] for j in range(NU)] for i in range(NX)])
        K: dict = {}
        rhs = [None] * n

        def put(i, j, v):
            if v is None:
                return
            if isinstance(v, float):
                v = g.const(v)
            if v.is_zero():
                return
            if i < j:
                i, j = j, i
            K[(i, j)] = v

        huu = []
        for k in range(T + 1):
            Qk = QTd if k == T else Qd
            for i in range(NX):
                put(ix[k] + i, ix[k] + i, Qk[i])
                rhs[ix[k] + i] = -(Qk[i] * xs[k][i])
            # constraint rows lam_k
            for i in range(NX):
                put(il[k] + i, ix[k] + i, 1.0)
                if k == 0:
                    rhs[il[k] + i] = xbar[i] - xs[0][i]
                else:
                    rhs[il[k] + i] = fk[k - 1][i] - xs[k][i]
                    for j in range(NX):
                        a = Ak[k - 1][i][j]
                        put(il[k] + i, ix[k - 1] + j, None if a is None else -a)
                    for j in range(NU):
                        b = Bk[k - 1][i][j]
                        put(il[k] + i, iu[k - 1] + j, None if b is None else -b)
            if k < T:
                u = us[k][0]
                pctx = g.precision(low)
                pctx.__enter__()
                if penalty:
                    h, grad = penalty_terms(u, umax, mu, R)
                else:
                    h = g.const(R)
                    grad = R * u
                pctx.__exit__(None, None, None)
                put(iu[k], iu[k], h)
                huu.append(h)
                rhs[iu[k]] = -grad
        sol, D = _ldl_solve(g, n, K, rhs)
        xs = [[xs[k][i] + sol[ix[k] + i] for i in range(NX)] for k in range(T + 1)]
        us = [[us[k][j] + sol[iu[k] + j] for j in range(NU)] for k in range(T)]
        mu = mu * alpha
        if outputs == "debug":
            dbg = dict(sol=sol, rhs=rhs, A=Ak, B=Bk, huu=huu, D=D, xlin=x_lin, ulin=u_lin)
    z = [v for k in range(T + 1) for v in xs[k]] + [v for k in range(T) for v in us[k]]
    if outputs == "z":
        return g.program([z], reuse_slots)
    if outputs == "debug":
        zero = g.const(0.0)
        Af = [(a if a is not None else zero) for Ak_ in dbg["A"] for r in Ak_ for a in r]
        Bf = [(b if b is not None else zero) for Bk_ in dbg["B"] for r in Bk_ for b in r]
        xl = [g.lift(v) for k in range(T) for v in dbg["xlin"][k]]
        ul = [g.lift(dbg["ulin"][k][0]) for k in range(T)]
        return g.program([z, dbg["sol"], dbg["rhs"], Af, Bf, dbg["huu"], dbg["D"], xl, ul], reuse_slots)
    raise ValueError(outputs)


def kkt_index(T: int):
    """(ix, il, iu) maps from stage to the first unknown of x_k, lam_k, u_k."""
    ix, il, iu = {}, {}, {}
    n = 0
    for k in range(T + 1):
        ix[k] = n
        n += NX
        il[k] = n
        n += NX
        if k < T:
            iu[k] = n
            n += NU
    return ix, il, iu, n


def cartpole_step(dt: float = 0.02, dtype: str = "f64", cp: CartPole | None = None):
    """One RK4 step of the cart-pole: inputs (x 4, u 1) -> x+ (4)."""
    cp = cp if cp is not None else CartPole()
    g = Graph("cartpole_rk4", dtype)
    x = g.input(NX)
    u = g.input(NU)
    return g.program([rk4(cp, x, u, dt)])
