"""Fill the on-disk kernel cache for the standard workloads (compile only:
no GPU is needed, hiprtc cross-compiles for gfx950).

    python -m paper_2408_09662_amd.warm [--all] [--batch] [--tune]

Without flags only the benchmark and smoke programs are compiled; --all adds
the other forward/adjoint modes, --batch the persistent launch of the
uneven-batch workload (three random DAGs of 1e3/1e4/1e5 operations and the
MPC), whose single code object takes minutes to build, --tune every
candidate the autotuner times for the benchmarked programs and instance
counts (forward, and the pendulum's adjoint).
"""

from __future__ import annotations

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BATCH_KEYS = ["rdag1e3", "rdag1e4", "rdag1e5", "mpc_b"]
TUNE_JOBS = [("rdag200", 1000), ("pend7", 16384), ("pend7", 65536), ("pend7_f32", 16384), ("pend7_f32", 65536),
             ("rdag1e4", 8192), ("mpc", 4096), ("mpc", 65536), ("mpc_mixed", 4096), ("mpc_mixed", 65536), ("mpc_m1", 4096),
             ("mpc_m2", 4096), ("mpc_m4", 4096), ("mpc_m5", 4096), ("quad", 10000)]
# adjoint plans the benchmark tunes (on the fused kernel) and then runs in
# both adjoint modes
ADJ_TUNE_JOBS = [("rdag200", 1000), ("pend7", 16384), ("pend7", 65536), ("pend7_f32", 65536)]
# cooperative-tile variants the tests and the benchmark evaluate
WIDE_JOBS = [("rdag200", 4), ("rdag200", 16), ("rdag1e4", 4), ("rdag1e4", 8), ("pend7", 2),
             ("pend7", 4), ("mpc", 4), ("rdag1e5", 8), ("rdag1e5", 16)]


def batch_programs():
    import paper_2408_09662_amd as xg
    from workloads import configs
    return [xg.Program(configs.program_path(k)) for k in BATCH_KEYS]


def coop_batch_programs():
    """The same four programs for one 512-lane persistent launch: the 1e5-op
    DAG as 8-wave cooperative tiles, the others on 512-lane workgroups."""
    import paper_2408_09662_amd as xg
    from workloads import configs
    return [xg.Program(configs.program_path(k), **({"waves": 8} if k == "rdag1e5" else {"block": 512}))
            for k in BATCH_KEYS]


def warm(all_programs: bool = False, batch: bool = False, tune: bool = False,
         verbose: bool = True) -> None:
    import paper_2408_09662_amd as xg
    from workloads import configs
    jobs = [("rdag200", (0, 1, 2)), ("pend7", (0, 2)), ("pend7_f32", (0,))]
    if all_programs:
        jobs += [("pend7", (1,)), ("pend7_f32", (1, 2)), ("mpc", (0,)), ("mpc_mixed", (0,))]
        jobs += [(k, (0,)) for k in BATCH_KEYS]
        jobs += [(k, (0,)) for k in configs.MPC_SWEEP if k != "mpc"]
        jobs += [(k, (0,)) for k in configs.LDL_SWEEP] + [("quad", (0,))]
    for key, modes in jobs:
        p = xg.Program(configs.program_path(key))
        for m in modes:
            t = time.time()
            p.precompile(m)
            if verbose:
                print(f"[warm] {key} mode {m}: {time.time() - t:.1f} s", flush=True)
    if all_programs:
        from workloads import probes
        for dt in ("f64", "f32"):
            xg.Program(probes.fma_chains(dtype=dt)).precompile(0)
        for key, w in WIDE_JOBS:
            t = time.time()
            xg.Program(configs.program_path(key), waves=w).precompile(0)
            if verbose:
                print(f"[warm] {key} waves {w}: {time.time() - t:.1f} s", flush=True)
    if tune:
        for key, n in TUNE_JOBS:
            t = time.time()
            xg.autotune_precompile(xg.Program(configs.program_path(key)), n)
            if verbose:
                print(f"[warm] tune candidates {key} n={n}: {time.time() - t:.1f} s", flush=True)
        for key, n in ADJ_TUNE_JOBS:
            t = time.time()
            for m in (2, 1):
                xg.autotune_precompile(xg.Program(configs.program_path(key)), n, m)
            if verbose:
                print(f"[warm] adjoint tune candidates {key} n={n}: {time.time() - t:.1f} s", flush=True)
    if batch:
        t = time.time()
        ps = batch_programs()
        xg.Batch(ps)
        if verbose:
            print(f"[warm] batch {'+'.join(BATCH_KEYS)}: {time.time() - t:.1f} s", flush=True)
        t = time.time()
        xg.Batch([p for k, p in zip(BATCH_KEYS, ps) if k != "rdag1e5"])
        if verbose:
            print(f"[warm] batch without rdag1e5: {time.time() - t:.1f} s", flush=True)
        t = time.time()
        xg.Batch(coop_batch_programs())
        if verbose:
            print(f"[warm] batch with cooperative tiles: {time.time() - t:.1f} s", flush=True)
        t = time.time()
        xg.autotune_batch_precompile(batch_programs(), [configs.ITEMS[k].n for k in BATCH_KEYS])
        if verbose:
            print(f"[warm] batch autotune candidates: {time.time() - t:.1f} s", flush=True)



if __name__ == "__main__":
    warm("--all" in sys.argv, "--batch" in sys.argv, "--tune" in sys.argv)
