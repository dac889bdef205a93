"""Fill the on-disk kernel cache for the standard workloads (compile only:
no GPU is needed, hiprtc cross-compiles for gfx950).

    python -m paper_2408_09662_amd.warm [--all]

Without --all only the benchmark and smoke programs are compiled.
"""

from __future__ import annotations

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def warm(all_programs: bool = False, verbose: bool = True) -> None:
    import paper_2408_09662_amd as xg
    from workloads import configs
    jobs = [("rdag200", (0, 1, 2)), ("pend7", (0, 2)), ("pend7_f32", (0,))]
    if all_programs:
        jobs += [("pend7", (1,)), ("pend7_f32", (1, 2)), ("mpc", (0,))]
    for key, modes in jobs:
        p = xg.Program(configs.program_path(key))
        for m in modes:
            t = time.time()
            p.precompile(m)
            if verbose:
                print(f"[warm] {key} mode {m}: {time.time() - t:.1f} s", flush=True)


if __name__ == "__main__":
    warm("--all" in sys.argv)
