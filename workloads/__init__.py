"""Workload construction shared by both sides of every parity check.

This package builds the straight-line scalar programs that are evaluated
(the paper's "work vector + instruction list" form, section "Code
Generation") and draws the seeded synthetic inputs.  It never evaluates a
program: it only records which operations are applied to which values.
The oracle (``oracle/``) and the GPU library (``paper_2408_09662_amd``)
both consume its output -- the program file and the input arrays -- and
share no other code.
"""

from .tracer import Graph, Sym, Program  # noqa: F401
