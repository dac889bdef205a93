"""Seeded random scalar DAGs (the synthetic stand-in for the paper's
benchmark functions, whose size grows by 10x per step).

Recipe (a reading; the workload description fixes the op set, the input
distribution U(-1, 1), the guards and the counts):

* the drawn operations are laid out in layers of width
  W = max(n_in, ceil(n_ops / depth)) with depth = 12, layer 0 being the
  inputs, so the graph is as deep for 1e5 ops as for 200 (with a first-in
  first-out chain of width n_in a 1e4-op graph is ~300 levels deep and so
  chaotic that long-double and double evaluations differ by O(1), which
  would make any parity tolerance meaningless);
* each operation is uniform over
  {ADD, SUB, MUL, DIVG, SIN, COS, EXPG, SQRTG, TANH};
* its first operand is the previous layer's value at the same position
  (cycling), so every value is consumed; a second operand is `pick()`:
  with probability 0.8 uniform over a window of 32 previous-layer values
  around that position (locality, as in real expression graphs), otherwise
  uniform over all values created before the current layer;
* guards are emitted as primitive instructions:
  DIVG(a, b) = a / (1 + |b|), EXPG(a) = exp(min(max(a, -5), 5)),
  SQRTG(a) = sqrt(1 + |a|);
* a drawn node is redrawn if its interval bound (propagated from the
  inputs' [-1, 1] by interval arithmetic on the structure, never by
  evaluating it) exceeds 1e6 in magnitude, or if a bound of its total input
  sensitivity sum_j |dv/dx_j| (chain rule with each op's derivative bounded
  over the operand intervals) exceeds 64, so every instance stays finite and
  the graph stays well conditioned (no chaotic error growth);
* the outputs are `n_out` pairwise sums over contiguous groups of the last
  layer, so no drawn operation is dead.
"""

from __future__ import annotations

import math
import random

from .tracer import Graph, sin, cos, tanh, exp, sqrt, fabs, fmin, fmax

OPS = ("ADD", "SUB", "MUL", "DIVG", "SIN", "COS", "EXPG", "SQRTG", "TANH")
BOUND = 1e6


def _ibound(op, ia, ib):
    lo, hi = ia
    if op == "ADD":
        return (lo + ib[0], hi + ib[1])
    if op == "SUB":
        return (lo - ib[1], hi - ib[0])
    if op == "MUL":
        ps = (lo * ib[0], lo * ib[1], hi * ib[0], hi * ib[1])
        return (min(ps), max(ps))
    if op == "DIVG":
        return (min(lo, 0.0), max(hi, 0.0))
    if op in ("SIN", "COS", "TANH"):
        return (-1.0, 1.0)
    if op == "EXPG":
        return (math.exp(max(min(lo, 5.0), -5.0)), math.exp(max(min(hi, 5.0), -5.0)))
    if op == "SQRTG":
        return (1.0, math.sqrt(1.0 + max(abs(lo), abs(hi))))
    raise ValueError(op)


def _gains(op, ia, ib):
    """Upper bounds of |d op / d a| and |d op / d b| over the operand intervals."""
    ma = max(abs(ia[0]), abs(ia[1]))
    if op in ("ADD", "SUB"):
        return 1.0, 1.0
    if op == "MUL":
        return max(abs(ib[0]), abs(ib[1])), ma
    if op == "DIVG":
        return 1.0, ma
    if op in ("SIN", "COS", "TANH"):
        return 1.0, 0.0
    if op == "EXPG":
        return math.exp(max(min(ia[1], 5.0), -5.0)), 0.0
    if op == "SQRTG":
        return 0.5, 0.0
    raise ValueError(op)


def rdag(seed: int, n_in: int = 8, n_ops: int = 200, n_out: int = 4,
         dtype: str = "f64", reuse_slots: bool = True, return_stats: bool = False,
         depth: int = 12, kappa_max: float = 64.0):
    rng = random.Random(seed)
    g = Graph(f"rdag_s{seed}_{n_in}x{n_ops}", dtype)
    xs = g.input(n_in)
    V = list(xs)
    iv = [(-1.0, 1.0)] * n_in
    kap = [1.0] * n_in  # bound of sum_j |d v / d x_j|
    W = max(n_in, -(-n_ops // depth))
    prev = list(range(n_in))   # indices into V of the previous layer
    cur: list[int] = []
    drawn = 0

    for t in range(n_ops):
        pos = t % W
        if pos == 0 and t > 0:
            prev, cur = cur, []
        ia = prev[pos % len(prev)]

        def pick():
            if rng.random() < 0.8:
                c = pos % len(prev)
                lo, hi = max(0, c - 16), min(len(prev), c + 16)
                return prev[rng.randrange(lo, hi)]
            return rng.randrange(0, prev[0] + len(prev)) if prev[0] > 0 else rng.choice(prev)

        for attempt in range(64):
            op = rng.choice(OPS)
            ib = pick() if op in ("ADD", "SUB", "MUL", "DIVG") else None
            bd = _ibound(op, iv[ia], iv[ib] if ib is not None else None)
            ga, gb = _gains(op, iv[ia], iv[ib] if ib is not None else None)
            kp = ga * kap[ia] + (gb * kap[ib] if ib is not None else 0.0)
            if max(abs(bd[0]), abs(bd[1])) <= BOUND and kp <= kappa_max:
                break
        else:  # bounded, contractive fallback
            op, ib, bd, kp = "SQRTG", None, _ibound("SQRTG", iv[ia], None), 0.5 * kap[ia]
        a = V[ia]
        if op == "ADD":
            r = a + V[ib]
        elif op == "SUB":
            r = a - V[ib]
        elif op == "MUL":
            r = a * V[ib]
        elif op == "DIVG":
            r = a / (1.0 + fabs(V[ib]))
        elif op == "SIN":
            r = sin(a)
        elif op == "COS":
            r = cos(a)
        elif op == "EXPG":
            r = exp(fmin(fmax(a, -5.0), 5.0))
        elif op == "SQRTG":
            r = sqrt(1.0 + fabs(a))
        else:
            r = tanh(a)
        drawn += 1
        V.append(r)
        iv.append(bd)
        kap.append(kp)
        cur.append(len(V) - 1)
    # every value of the last layer (and any previous-layer value a partial
    # last layer did not consume) feeds an output: the n_out outputs are
    # pairwise-summed groups of them, so no drawn operation is dead code
    final = cur + prev[len(cur):]
    outs = []
    for k in range(n_out):
        grp = [V[i] for i in final[k * len(final) // n_out:(k + 1) * len(final) // n_out]]
        if not grp:
            grp = [V[final[-1 - k]]]
        while len(grp) > 1:
            nxt = [grp[i] + grp[i + 1] for i in range(0, len(grp) - 1, 2)]
            if len(grp) % 2:
                nxt.append(grp[-1])
            grp = nxt
        outs.append(grp[0])
    prog = g.program([outs], reuse_slots)
    if return_stats:
        return prog, {"drawn": drawn, "emitted": prog.n_arith(), "width": W}
    return prog
