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
