"""Benchmark: instance evaluations per second of the straight-line program
evaluator on one MI355X, with the roofline of its kernel and the oracle's
CPU rate beside it.

Workload (the headline configuration): one RK4 step (dt = 1e-3) of the
planar 7-link pendulum -- mass matrix, Christoffel Coriolis term, gravity,
unrolled 7x7 Cholesky solve -- as one straight-line fp64 program of 15,354
scalar operations, evaluated for N = 16,384 independent instances whose
inputs already sit in HBM (structure of arrays, seeded synthetic states:
q ~ U(-pi, pi), qdot ~ N(0, 1)).  A step is one evaluation of all N
instances.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Secondary figures (the same program at N = 65,536,
fp32, the fused forward+adjoint, the MPC) are reported under "secondary".
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12   # MI355X FP64 vector FLOP/s (FMA = 2)
PEAK_FP32 = 157.3e12  # MI355X FP32 vector FLOP/s (packed)
PEAK_HBM = 8.0e12     # bytes/s


def _ops_per_instance(path):
    import paper_2408_09662_amd as xg
    d = xg.load_program_file(path)
    data_ops = {xg.OP_ID[k] for k in ("INPUT", "OUTPUT", "CONST", "ASSIGN")}
    return int(sum(1 for op in d["instr"][:, 0] if int(op) not in data_ops))


def time_eval(prog, xin, steps, warmup, stream=None):
    """Average seconds per evaluation, HIP events on the launch stream."""
    import torch
    n = xin[0].shape[1]
    outs = prog.alloc_outputs(n)
    ws = prog.workspace(n, 0)
    s = torch.cuda.current_stream() if stream is None else stream
    run = prog.bind_eval(xin, outs, workspace=ws, stream=s)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        run()
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) * 1e-3 / steps, wall


def time_adjoint(prog, xin, seeds, steps, warmup, fused=True):
    import torch
    n = xin[0].shape[1]
    grads = [torch.empty((k, n), dtype=prog.torch_dtype, device="cuda") for k in prog.nnz_in]
    outs = prog.alloc_outputs(n) if fused else None
    ws = prog.workspace(n, 2 if fused else 1)
    for _ in range(warmup):
        prog.eval_adjoint(xin, seeds, grads=grads, outputs=outs, with_outputs=fused, workspace=ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        prog.eval_adjoint(xin, seeds, grads=grads, outputs=outs, with_outputs=fused, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / steps


def bench_batch(steps):
    """Workload 5: three random DAGs (1e3/1e4/1e5 drawn ops, fp32, N = 65,536 /
    8,192 / 512) and the MPC (fp64, N = 2,048) -- one persistent launch vs the
    four programs' own kernels launched back to back, and graph replay."""
    import torch
    import paper_2408_09662_amd as xg
    from workloads import configs
    keys = ["rdag1e3", "rdag1e4", "rdag1e5", "mpc_b"]
    progs = [xg.Program(configs.program_path(k)) for k in keys]
    xin = []
    for k, p in zip(keys, progs):
        xin.append([torch.from_numpy(x).to(p.torch_dtype).cuda() for x in configs.item_inputs(k)])
    outs = [p.alloc_outputs(x[0].shape[1]) for p, x in zip(progs, xin)]
    b = xg.Batch(progs)
    ntot = sum(x[0].shape[1] for x in xin)
    steps = max(5, steps // 5)

    def timed(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    runs = [p.bind_eval(x, o) for p, x, o in zip(progs, xin, outs)]
    t_seq = timed(lambda: [r() for r in runs], steps)
    ws = b.workspace([x[0].shape[1] for x in xin])
    t_batch = timed(lambda: b.eval(xin, outs, workspace=ws), steps)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = b.capture(xin, outs, stream=s, workspace=ws)
        t_graph = timed(lambda: g.launch(stream=s), steps)
    return {"instances": ntot, "sequential_ms": t_seq * 1e3, "persistent_ms": t_batch * 1e3,
            "persistent_graph_ms": t_graph * 1e3,
            "instance_evals_per_s_persistent": ntot / t_batch}


def cpu_baseline(path, x, min_seconds=3.0):
    """The oracle (test infrastructure) on the host cores: double precision
    interpreter over the same program and inputs."""
    from oracle.pyoracle import Program as OProg
    o = OProg(path)
    threads = max(1, min(os.cpu_count() or 1, 16))
    n = x.shape[1]
    reps = 0
    t0 = time.perf_counter()
    while True:
        o.evaluate([x], 64, threads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    return {"value": reps * n / el, "unit": "instance-evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"full workload ({n} instances, fp64 interpreter) x {reps} repetitions, "
                      f"{el:.1f} s wall on {threads} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the persistent-batch figures")
    ap.add_argument("--n", type=int, default=0,
                    help="instances (default: the workload's 16,384); for profiling other sizes")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this evaluator runs on one GPU; multi-GPU runs are not part of this "
              "build (instances shard with no communication: see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        nb = args.copy_calibration << 20
        a = torch.empty(nb // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": nb, "launches": 5}))
        return
    import paper_2408_09662_amd as xg
    from workloads import configs

    key = "pend7"
    it = configs.ITEMS[key]
    path = configs.program_path(key)
    n = args.n if args.n > 0 else it.n
    x = it.make_inputs(n)[0]
    prog = xg.Program(path)
    xin = [torch.from_numpy(x).cuda()]
    prog.compile(0)
    sec, wall = time_eval(prog, xin, args.steps, args.warmup)
    ops = _ops_per_instance(path)
    flops = ops * n
    nbytes = (14 + 14) * 8 * n
    achieved = flops / sec
    value = n / sec
    out = {
        "metric": "instance-evals/s and % FP64-VALU/HBM roofline, forward and fwd+adjoint, 1 GPU",
        "value": value,
        "unit": "instance-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded pendulum states, inputs resident in HBM)",
        "config": {"workload": "pendulum7_rk4_fwd", "n_instances": n, "ops_per_instance": ops,
                   "program": "7-link planar pendulum, one RK4 step dt=1e-3, fp64"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                     "kernel": "xg_m0_c0 (pendulum RK4 forward)",
                     "algorithmic_flops_per_launch": flops,
                     "algorithmic_bytes_per_launch": nbytes},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(path, x)
    if not args.no_secondary:
        sec2 = {}
        steps2 = max(20, args.steps // 10)
        # same program at 4x the instances (fills every SIMD once)
        x4 = configs.ITEMS["pend7_grad"].make_inputs(65536)[0]
        s4, _ = time_eval(prog, [torch.from_numpy(x4).cuda()], steps2, 5)
        sec2["pendulum7_fwd_f64_n65536"] = {"instance_evals_per_s": 65536 / s4,
                                            "frac_fp64": ops * 65536 / s4 / PEAK_FP64}
        p32 = xg.Program(configs.program_path("pend7_f32"))
        s32, _ = time_eval(p32, [torch.from_numpy(x).float().cuda()], steps2, 5)
        sec2["pendulum7_fwd_f32_n16384"] = {"instance_evals_per_s": n / s32,
                                            "frac_fp32": ops * n / s32 / PEAK_FP32}
        try:
            ya = torch.from_numpy(2.0 * x).cuda()
            sa = time_adjoint(prog, xin, [ya], steps2, 5, fused=True)
            sec2["pendulum7_fused_fwd_adjoint_f64_n16384"] = {"instance_evals_per_s": n / sa,
                                                              "ratio_to_forward": sa / sec}
        except Exception as e:  # noqa: BLE001
            sec2["pendulum7_fused_fwd_adjoint_f64_n16384"] = {"error": str(e)[:200]}
        try:
            pm = xg.Program(configs.program_path("mpc"))
            xm = configs.item_inputs("mpc")[0]
            sm, _ = time_eval(pm, [torch.from_numpy(xm).cuda()], max(10, steps2 // 4), 3)
            sec2["cartpole_mpc_f64_n4096"] = {"instance_evals_per_s": 4096 / sm,
                                              "ms_per_eval": sm * 1e3}
        except Exception as e:  # noqa: BLE001
            sec2["cartpole_mpc_f64_n4096"] = {"error": str(e)[:200]}
        if not args.no_batch:
            try:
                sec2["uneven_batch"] = bench_batch(steps2)
            except Exception as e:  # noqa: BLE001
                sec2["uneven_batch"] = {"error": str(e)[:300]}
        out["secondary"] = sec2
    print(json.dumps(out))


if __name__ == "__main__":
    main()
