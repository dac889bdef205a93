"""Probe programs for measuring what the chip reaches through this code
generator: not workloads of the paper, only references for the measured
fractions (the vendor peaks stay the denominators).

fma_chains: `chains` independent recurrences v <- v*a + b of `length`
steps each (the compiler contracts every step into one FMA), so an
instance issues chains*length FMAs with `chains`-way instruction-level
parallelism and almost no memory traffic.
"""

from __future__ import annotations

from .tracer import Graph


def fma_chains(chains: int = 8, length: int = 1024, dtype: str = "f64"):
    g = Graph(f"fma{chains}x{length}_{dtype}", dtype)
    x = g.input(chains)
    a = g.const(0.999999)
    b = g.const(1e-6)
    outs = []
    for c in range(chains):
        v = x[c]
        for _ in range(length):
            v = v * a + b
        outs.append(v)
    return g.program([outs])


def fma_flops(chains: int = 8, length: int = 1024) -> int:
    """FLOPs per instance, an FMA counted as two."""
    return 2 * chains * length


def copy(n_in: int = 1, n_out: int | None = None, dtype: str = "f64"):
    """y[e] = x[e mod n_in] for e < n_out: every element one coalesced load
    and one coalesced store through the generated access helpers (the same
    access width as any program's inputs and outputs), no arithmetic.  With
    n_out = n_in it moves exactly (n_in reads + n_in writes) x element size
    per instance; with n_in = 8, n_out = 4 it has the random DAG's argument
    shapes (the launch floor of a program of that size)."""
    n_out = n_in if n_out is None else n_out
    g = Graph(f"copy{n_in}x{n_out}_{dtype}", dtype)
    x = g.input(n_in)
    return g.program([[x[e % n_in] for e in range(n_out)]])
