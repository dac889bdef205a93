"""Expression tracer: records scalar programs as a DAG of unary/binary ops.

The program model is the one of the paper's background section on SX
graphs: every closed-form expression is a finite sequence of atomic unary
(R -> R) and binary (R x R -> R) scalar operations, and matrix algebra is
expanded into those.  A :class:`Graph` records the operations applied to
:class:`Sym` handles (with hash-consing, so identical sub-expressions are
recorded once) and lowers the result to a :class:`Program`: a work vector
plus an instruction list (section "Code Generation"), with inputs and
outputs given as dense vectors of structural non-zeros.

Nothing here evaluates floating-point values.  The only simplifications are
structural identities (x+0, x*1, x*0, --x, ...), which CasADi applies as
well, and they never change a finite result.
"""

from __future__ import annotations

import struct

# Opcode table: name -> arity.  INPUT/OUTPUT/CONST are the data movement
# ops; ASSIGN copies a slot.  The set is the one listed in the paper's
# mapping table plus the unary/binary functions its text names (log, cos,
# sqrt, atan2, min/max) and a few that the workloads need.
ARITY = {
    "INPUT": 0, "OUTPUT": 1, "CONST": 0, "ASSIGN": 1,
    "ADD": 2, "SUB": 2, "MUL": 2, "DIV": 2,
    "NEG": 1, "SQ": 1, "SQRT": 1, "EXP": 1, "LOG": 1,
    "SIN": 1, "COS": 1, "TAN": 1, "TANH": 1, "ATAN": 1,
    "FABS": 1, "FMIN": 2, "FMAX": 2, "LT": 2, "LE": 2,
    "POW": 2, "ATAN2": 2,
}
COMMUTATIVE = {"ADD", "MUL"}


def _fbits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", float(x)))[0]


class Graph:
    """A DAG of scalar operations; node i depends only on nodes < i."""

    def __init__(self, name: str = "prog", dtype: str = "f64"):
        if dtype not in ("f64", "f32"):
            raise ValueError("dtype must be f64 or f32")
        self.name = name
        self.dtype = dtype
        self.op: list[str] = []
        self.a: list[int] = []
        self.b: list[int] = []
        self.aux: list = []
        self._memo: dict = {}
        self.nnz_in: list[int] = []
        self.inputs: list[list[Sym]] = []
        self.prec: list = []     # per node: None (program dtype) or "f32"
        self._prec_now = None

    # -- node creation -------------------------------------------------
    def _node(self, op: str, a: int = -1, b: int = -1, aux=None) -> int:
        if op in COMMUTATIVE and a > b:
            a, b = b, a
        prec = self._prec_now if op not in ("INPUT", "CONST") else None
        key = (op, a, b, aux, prec)
        i = self._memo.get(key)
        if i is not None:
            return i
        i = len(self.op)
        self.op.append(op)
        self.a.append(a)
        self.b.append(b)
        self.aux.append(aux)
        self.prec.append(prec)
        self._memo[key] = i
        return i

    class _Precision:
        def __init__(self, g, prec):
            self.g, self.prec = g, prec

        def __enter__(self):
            self.old = self.g._prec_now
            self.g._prec_now = self.prec
            return self

        def __exit__(self, *a):
            self.g._prec_now = self.old

    def precision(self, prec):
        """Context: operations recorded inside are tagged with `prec`
        ("f32" inside an f64 program: operands rounded to binary32, the
        operation done in binary32, the result widened exactly)."""
        if prec not in (None, "f32"):
            raise ValueError("only f32 instructions can be tagged (in an f64 program)")
        if prec is not None and self.dtype != "f64":
            raise ValueError("precision tags need an f64 program")
        return Graph._Precision(self, prec)

    def const(self, v: float) -> "Sym":
        v = float(v)
        return Sym(self, self._node("CONST", aux=("c", _fbits(v), v)))

    def input(self, nnz: int) -> list["Sym"]:
        """Declare a new input argument with `nnz` scalar entries."""
        arg = len(self.nnz_in)
        self.nnz_in.append(nnz)
        xs = [Sym(self, self._node("INPUT", aux=("i", arg, k))) for k in range(nnz)]
        self.inputs.append(xs)
        return xs

    # -- helpers ------------------------------------------------------
    def is_const(self, i: int, v: float | None = None) -> bool:
        if self.op[i] != "CONST":
            return False
        return v is None or self.aux[i][2] == v

    def const_value(self, i: int) -> float:
        return self.aux[i][2]

    def lift(self, x) -> "Sym":
        if isinstance(x, Sym):
            if x.g is not self:
                raise ValueError("mixing graphs")
            return x
        return self.const(x)

    def apply(self, op: str, x, y=None) -> "Sym":
        """Record `op` on operands, applying structural identities."""
        xs = self.lift(x)
        a = xs.i
        if ARITY[op] == 1:
            if op == "NEG":
                if self.op[a] == "NEG":
                    return Sym(self, self.a[a])
                if self.is_const(a):
                    return self.const(-self.const_value(a))  # exact sign flip
            return Sym(self, self._node(op, a))
        ys = self.lift(y)
        b = ys.i
        z0 = lambda i: self.is_const(i) and self.const_value(i) == 0.0  # noqa: E731
        o1 = lambda i: self.is_const(i, 1.0)  # noqa: E731
        if op == "ADD":
            if z0(a):
                return ys
            if z0(b):
                return xs
        elif op == "SUB":
            if z0(b):
                return xs
            if z0(a):
                return self.apply("NEG", ys)
        elif op == "MUL":
            if z0(a) or z0(b):
                return self.const(0.0)
            if o1(a):
                return ys
            if o1(b):
                return xs
            if self.is_const(a, -1.0):
                return self.apply("NEG", ys)
            if self.is_const(b, -1.0):
                return self.apply("NEG", xs)
        elif op == "DIV":
            if o1(b):
                return xs
            if z0(a):
                return self.const(0.0)
        return Sym(self, self._node(op, a, b))

    # -- lowering -----------------------------------------------------
    def program(self, outputs: list[list["Sym"]], reuse_slots: bool = True) -> "Program":
        """Lower to a work-vector program computing `outputs` (list of args)."""
        outs = [[self.lift(s).i for s in arg] for arg in outputs]
        n = len(self.op)
        need = bytearray(n)
        stack = [i for arg in outs for i in arg]
        while stack:
            i = stack.pop()
            if need[i]:
                continue
            need[i] = 1
            if self.a[i] >= 0:
                stack.append(self.a[i])
            if self.b[i] >= 0:
                stack.append(self.b[i])
        order = [i for i in range(n) if need[i]]
        # last use of each node (OUTPUT uses count as the end of the program)
        end = len(order)
        last = {}
        for t, i in enumerate(order):
            for j in (self.a[i], self.b[i]):
                if j >= 0:
                    last[j] = t
        for arg in outs:
            for i in arg:
                last[i] = end
        consts: list[float] = []
        cidx: dict = {}
        slot: dict = {}
        free: list[int] = []
        n_work = 0
        instrs: list[tuple[str, int, int, int]] = []
        precs: dict = {}
        for t, i in enumerate(order):
            op = self.op[i]
            if reuse_slots:
                for j in {self.a[i], self.b[i]}:
                    if j >= 0 and last[j] == t:
                        free.append(slot[j])
            if reuse_slots and free:
                s = free.pop()
            else:
                s = n_work
                n_work += 1
            if op == "INPUT":
                instrs.append(("INPUT", s, self.aux[i][1], self.aux[i][2]))
            elif op == "CONST":
                key = self.aux[i][1]
                if key not in cidx:
                    cidx[key] = len(consts)
                    consts.append(self.aux[i][2])
                instrs.append(("CONST", s, cidx[key], -1))
            else:
                a = slot[self.a[i]]
                b = slot[self.b[i]] if self.b[i] >= 0 else -1
                if self.prec[i] is not None:
                    precs[len(instrs)] = self.prec[i]
                instrs.append((op, s, a, b))
            slot[i] = s
            if reuse_slots and last.get(i, -1) == -1:
                free.append(s)  # defined but never used (cannot happen after DCE)
        for k, arg in enumerate(outs):
            for nz, i in enumerate(arg):
                instrs.append(("OUTPUT", k, slot[i], nz))
        return Program(
            name=self.name, dtype=self.dtype, n_work=max(n_work, 1),
            nnz_in=list(self.nnz_in), nnz_out=[len(a) for a in outs],
            consts=consts, instrs=instrs, prec=precs,
        )

    # -- symbolic forward-mode differentiation ------------------------
    def jacobian(self, ys: list["Sym"], xs: list["Sym"]) -> list[list["Sym | None"]]:
        """J[i][j] = d ys[i] / d xs[j] as Syms (None = structural zero)."""
        yi = [self.lift(y).i for y in ys]
        xi = [self.lift(x).i for x in xs]
        hi = max(yi) if yi else -1
        lo = min(xi) if xi else 0
        xset = set(xi)
        cols = []
        for x in xi:
            tan: dict[int, Sym] = {x: self.const(1.0)}
            for i in range(lo, hi + 1):
                if i == x:
                    continue
                a, b = self.a[i], self.b[i]
                ta = tan.get(a) if a >= 0 else None
                tb = tan.get(b) if b >= 0 else None
                if ta is None and tb is None:
                    continue
                if i in xset:
                    raise ValueError("jacobian: one independent variable depends on another")
                d = self._tangent(i, ta, tb)
                if d is not None and not d.is_zero():
                    tan[i] = d
            cols.append([tan.get(y) for y in yi])
        return [[cols[j][i] for j in range(len(xi))] for i in range(len(yi))]

    def _tangent(self, i: int, ta, tb):
        """Tangent of node i given operand tangents (None = zero)."""
        op = self.op[i]
        A = Sym(self, self.a[i])
        B = Sym(self, self.b[i]) if self.b[i] >= 0 else None
        V = Sym(self, i)

        def acc(u, v):
            if u is None:
                return v
            if v is None:
                return u
            return u + v

        if op == "ADD":
            return acc(ta, tb)
        if op == "SUB":
            return acc(ta, None if tb is None else -tb)
        if op == "MUL":
            return acc(None if ta is None else ta * B, None if tb is None else A * tb)
        if op == "DIV":
            u = None if ta is None else ta / B
            v = None if tb is None else -(tb * V) / B
            return acc(u, v)
        if op == "NEG":
            return -ta
        if op == "ASSIGN":
            return ta
        if op == "SQ":
            return ta * (2.0 * A)
        if op == "SQRT":
            return ta / (2.0 * V)
        if op == "EXP":
            return ta * V
        if op == "LOG":
            return ta / A
        if op == "SIN":
            return ta * cos(A)
        if op == "COS":
            return -(ta * sin(A))
        if op == "TAN":
            return ta * (1.0 + V * V)
        if op == "TANH":
            return ta * (1.0 - V * V)
        if op == "ATAN":
            return ta / (1.0 + A * A)
        if op in ("LT", "LE"):
            return None
        raise NotImplementedError(f"tracer derivative of {op}")


class Sym:
    """Handle of a node in a :class:`Graph` with arithmetic overloads."""

    __slots__ = ("g", "i")

    def __init__(self, g: Graph, i: int):
        self.g = g
        self.i = i

    def __add__(self, o):
        return self.g.apply("ADD", self, o)

    def __radd__(self, o):
        return self.g.apply("ADD", o, self)

    def __sub__(self, o):
        return self.g.apply("SUB", self, o)

    def __rsub__(self, o):
        return self.g.apply("SUB", o, self)

    def __mul__(self, o):
        return self.g.apply("MUL", self, o)

    def __rmul__(self, o):
        return self.g.apply("MUL", o, self)

    def __truediv__(self, o):
        return self.g.apply("DIV", self, o)

    def __rtruediv__(self, o):
        return self.g.apply("DIV", o, self)

    def __neg__(self):
        return self.g.apply("NEG", self)

    def is_zero(self) -> bool:
        return self.g.is_const(self.i) and self.g.const_value(self.i) == 0.0


class Dual:
    """Forward-mode dual number over Syms: value and tangent Syms.

    Used to form Jacobians of a sub-expression at the current iterate
    without treating the iterate's components as leaves: a tangent is
    carried explicitly, so a structural simplification of the value (for
    instance u = 0 making F*c vanish) never drops a derivative term.
    Tangent entries are Syms or None (structural zero)."""

    __slots__ = ("v", "d")

    def __init__(self, v, d):
        self.v = v
        self.d = d

    @staticmethod
    def _add(x, y):
        if x is None:
            return y
        if y is None:
            return x
        return x + y

    @staticmethod
    def _scale(x, c):
        return None if x is None else x * c

    def _lift(self, o):
        if isinstance(o, Dual):
            return o
        return Dual(o, [None] * len(self.d))

    def __add__(self, o):
        o = self._lift(o)
        return Dual(self.v + o.v, [Dual._add(a, b) for a, b in zip(self.d, o.d)])

    __radd__ = __add__

    def __sub__(self, o):
        o = self._lift(o)
        return Dual(self.v - o.v, [Dual._add(a, None if b is None else -b) for a, b in zip(self.d, o.d)])

    def __rsub__(self, o):
        return self._lift(o) - self

    def __mul__(self, o):
        o = self._lift(o)
        return Dual(self.v * o.v, [Dual._add(Dual._scale(a, o.v), Dual._scale(b, self.v))
                                   for a, b in zip(self.d, o.d)])

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = self._lift(o)
        q = self.v / o.v
        return Dual(q, [Dual._add(None if a is None else a / o.v,
                                  None if b is None else -(b * q) / o.v)
                        for a, b in zip(self.d, o.d)])

    def __rtruediv__(self, o):
        return self._lift(o) / self

    def __neg__(self):
        return Dual(-self.v, [None if a is None else -a for a in self.d])

    def unary(self, op):
        v = self.v.g.apply(op, self.v)
        if op == "SIN":
            dv = cos(self.v)
        elif op == "COS":
            dv = -sin(self.v)
        elif op == "SQRT":
            dv = 0.5 / v
        elif op == "EXP":
            dv = v
        elif op == "TANH":
            dv = 1.0 - v * v
        elif op == "SQ":
            dv = 2.0 * self.v
        else:
            raise NotImplementedError(op)
        return Dual(v, [Dual._scale(a, dv) for a in self.d])

    @staticmethod
    def seed(vals):
        """Duals for independent variables `vals` (one tangent direction each)."""
        k = len(vals)
        out = []
        for i, x in enumerate(vals):
            g = x.g if isinstance(x, Sym) else None
            d = [None] * k
            d[i] = g.const(1.0) if g is not None else 1.0
            out.append(Dual(x, d))
        return out


def _u(op):
    def f(x):
        if isinstance(x, Dual):
            return x.unary(op)
        return x.g.apply(op, x)
    f.__name__ = op.lower()
    return f


sin, cos, tan, tanh, atan = _u("SIN"), _u("COS"), _u("TAN"), _u("TANH"), _u("ATAN")
exp, log, sqrt, fabs, sq = _u("EXP"), _u("LOG"), _u("SQRT"), _u("FABS"), _u("SQ")


def fmin(x, y):
    g = x.g if isinstance(x, Sym) else y.g
    return g.apply("FMIN", x, y)


def fmax(x, y):
    g = x.g if isinstance(x, Sym) else y.g
    return g.apply("FMAX", x, y)


def lt(x, y):
    g = x.g if isinstance(x, Sym) else y.g
    return g.apply("LT", x, y)


class Program:
    """A work-vector program: the unit both evaluators consume.

    Instruction fields ``(op, out, a, b)``:
      INPUT  out=slot, a=arg, b=nz        CONST out=slot, a=constant index
      OUTPUT out=arg,  a=src slot, b=nz   unary  out=slot, a=src
      binary out=slot, a, b = source slots
    Semantics are sequential: each instruction reads its operands, then
    writes its output slot (so ``out`` may equal ``a`` or ``b``).  In an f64
    program, instructions listed in ``prec`` as "f32" round their operands to
    binary32, compute in binary32 and store the (exactly widened) result.
    """

    def __init__(self, name, dtype, n_work, nnz_in, nnz_out, consts, instrs, prec=None):
        self.name = name
        self.dtype = dtype
        self.n_work = n_work
        self.nnz_in = list(nnz_in)
        self.nnz_out = list(nnz_out)
        self.consts = list(consts)
        self.instrs = list(instrs)
        # instruction index -> "f32" for instructions computed in binary32
        self.prec = dict(prec or {})

    def op_counts(self) -> dict:
        c: dict = {}
        for ins in self.instrs:
            c[ins[0]] = c.get(ins[0], 0) + 1
        return c

    def n_arith(self) -> int:
        """Arithmetic instructions (everything but data movement)."""
        return sum(v for k, v in self.op_counts().items()
                   if k not in ("INPUT", "OUTPUT", "CONST", "ASSIGN"))

    def as_dtype(self, dtype: str) -> "Program":
        return Program(self.name, dtype, self.n_work, self.nnz_in, self.nnz_out,
                       self.consts, self.instrs, self.prec if dtype == "f64" else None)

    def text(self) -> str:
        out = [
            "xgprog 1",
            f"name {self.name}",
            f"dtype {self.dtype}",
            f"n_work {self.n_work}",
            "inputs " + " ".join([str(len(self.nnz_in))] + [str(k) for k in self.nnz_in]),
            "outputs " + " ".join([str(len(self.nnz_out))] + [str(k) for k in self.nnz_out]),
            f"consts {len(self.consts)}",
        ]
        out += [float(c).hex() for c in self.consts]
        out.append(f"instrs {len(self.instrs)}")
        out += [f"{o} {p} {a} {b}" for (o, p, a, b) in self.instrs]
        if self.prec:
            out.append(f"prec {len(self.prec)}")
            out += [f"{i} {v}" for i, v in sorted(self.prec.items())]
        out.append("end")
        return "\n".join(out) + "\n"

    def save(self, path) -> None:
        with open(path, "w") as f:
            f.write(self.text())


def worked_example() -> Program:
    """f(x) = (sin x + x)^2 written with the slot reuse of the paper's
    generated-kernel listing: slot 1 is both operand and result twice."""
    return Program(
        name="worked_example", dtype="f64", n_work=2, nnz_in=[1], nnz_out=[1],
        consts=[],
        instrs=[("INPUT", 0, 0, 0), ("SIN", 1, 0, -1), ("ADD", 1, 1, 0),
                ("MUL", 1, 1, 1), ("OUTPUT", 0, 1, 0)],
    )
