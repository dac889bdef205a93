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
PEAK_ISSUE = 39.3e12  # VALU lane-instructions/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz

# HBM traffic of the headline kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# (KiB per dispatch), each scaled by what the same counter reads for the
# copy probe (workloads/probes.copy: one 8-byte load and one 8-byte store
# per lane and element, the access width of every program argument) of a
# known size (`--copy-calibration`); valid only for the kernels with these
# code hashes at N = 16,384 (profiles/pendulum7_fwd_f64_n16384_traffic.txt).
# The autotuner's two closest plans (phases of about 300 and 150 cost units,
# within 2 % of each other) are both profiled, since either may win on a
# given box.
PROFILED_N = 16384
PROFILED_TRAFFIC = {0x98df90b6b59380d7: 4358144 + 1835008, 0x12757324967a6dc6: 4382720 + 1835008}
# FP64 FLOPs the hardware executed per launch of the same kernel, from
# rocprofv3 SQ_INSTS_VALU_FLOPS_FP64 (FLOPs per wave instruction, an FMA as
# two) x 64 lanes (profiles/pendulum7_fwd_f64_flop_counters.txt).
PROFILED_FLOPS = {0x98df90b6b59380d7: 6409728 * 64, 0x12757324967a6dc6: 6433024 * 64}

# The paper's own speed-ups (Table I; Intel i7-10850K CPU + NVIDIA RTX 3090
# GPU, fp64, batch 4,096 / 4,096 / 10,000): GPU over parallel CPU evaluation
# with host<->device transfer [and without].  Context only: other hardware,
# other functions, a CPU path that is not this oracle.
PAPER_TABLE_I = {
    "hardware": "Intel i7-10850K + NVIDIA RTX 3090 (the paper's benchmark machine)",
    "humanoid_srbm_mpc_1e5_instr_batch4096": {"with_transfer": 14.38, "compute_only": 1.54},
    "centroidal_momentum_1e4_instr_batch4096": {"with_transfer": 104.84, "compute_only": 1.98},
    "quadcopter_lqr_1e4_instr_batch10000": {"with_transfer": 143.18, "compute_only": 2.98},
}


def _ops_per_instance(path):
    import paper_2408_09662_amd as xg
    d = xg.load_program_file(path)
    data_ops = {xg.OP_ID[k] for k in ("INPUT", "OUTPUT", "CONST", "ASSIGN")}
    return int(sum(1 for op in d["instr"][:, 0] if int(op) not in data_ops))


def _plan_of(prog, tuned, mode=0):
    keys = ("block", "ipt", "reg_budget", "lds_slots", "prefetch", "chunk_ops", "waves", "coop_phase")
    if mode != 0:
        keys += ("adj_seg_ops",)
    o = prog.effective_options(mode)
    return {"autotuned": tuned is not None, **{k: o[k] for k in keys}}


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


def achievable_peaks(steps):
    """What the chip reaches here: FP64 and (unpacked) FP32 FMA issue through
    this code generator (probe programs of 8 independent 1,024-step FMA
    recurrences at 262,144 instances, four waves per SIMD) and a device-to-
    device copy of 1 GiB (read + write bytes over time)."""
    import torch
    import paper_2408_09662_amd as xg
    from workloads import probes
    res = {}
    n = 262144
    for dt, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        p = xg.Program(probes.fma_chains(dtype=dt))
        x = torch.rand((8, n), dtype=tdt, device="cuda")
        t, _ = time_eval(p, [x], steps, 3)
        res[f"{dt}_fma_tflops"] = probes.fma_flops() * n / t / 1e12
    nb = 1 << 30
    a = torch.empty(nb // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    res["hbm_copy_tbps"] = 2 * nb / (e0.elapsed_time(e1) * 1e-3 / 10) / 1e12
    return res


def launch_spread(prog, xin, launches):
    """Median and minimum of single-launch durations (an event pair around
    each launch on the launch stream)."""
    import torch
    n = xin[0].shape[1]
    outs = prog.alloc_outputs(n)
    ws = prog.workspace(n, 0)
    s = torch.cuda.current_stream()
    run = prog.bind_eval(xin, outs, workspace=ws, stream=s)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(launches)]
    for _ in range(5):
        run()
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(s)
        run()
        b.record(s)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    return {"median_ms": ms[len(ms) // 2], "min_ms": ms[0], "launches": launches}


def bench_reverse_mode(steps, tune=True):
    """Workload 4: the gradient of the final state's squared norm with respect
    to the 14 initial states at 65,536 instances, fp64 and fp32, through
    torch.autograd (forward kernel, then the adjoint kernel that recomputes
    the forward values it needs), next to the fused forward+adjoint kernel
    and the forward alone (forward plan and adjoint plan autotuned)."""
    import torch
    import paper_2408_09662_amd as xg
    from workloads import configs
    res = {}
    for key, tag in (("pend7_grad", "f64"), ("pend7_grad_f32", "f32")):
        p = xg.Program(configs.program_path(key))
        x = configs.item_inputs(key)[0]
        n = x.shape[1]
        xt = torch.from_numpy(x).to(p.torch_dtype).cuda()
        fplan = xg.autotune(p, [xt]) if tune else None
        aplan = xg.autotune_adjoint(p, [xt], [2.0 * p.eval([xt])[0]], fused=True) if tune else None
        xr = xt.clone().requires_grad_(True)

        def step():
            xr.grad = None
            y = xg.XgFunction.apply(p, xr)
            (y * y).sum().backward()

        for _ in range(3):
            step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        t_ag = e0.elapsed_time(e1) * 1e-3 / steps
        t_fwd, _ = time_eval(p, [xt], steps, 3)
        ys = p.eval([xt])[0]
        t_fused = time_adjoint(p, [xt], [2.0 * ys], steps, 3, fused=True)
        res[tag] = {"autograd_fwd_bwd_ms": t_ag * 1e3,
                    "instance_evals_per_s_autograd": n / t_ag,
                    "fused_kernel_ms": t_fused * 1e3,
                    "instance_evals_per_s_fused": n / t_fused,
                    "forward_ms": t_fwd * 1e3,
                    "autograd_to_forward": t_ag / t_fwd,
                    "fused_to_forward": t_fused / t_fwd,
                    "plan": _plan_of(p, fplan),
                    "adjoint_plan": _plan_of(p, aplan, mode=2)}
    return res


def bench_batch(steps):
    """Workload 5: three random DAGs (1e3/1e4/1e5 drawn ops, fp32, N = 65,536 /
    8,192 / 512) and the MPC (fp64, N = 2,048) -- the four programs' own
    kernels launched back to back vs one persistent launch (and its graph
    replay) on 64-lane workgroups, vs two concurrent launches, vs one
    persistent launch on 512-lane workgroups holding the 1e5-op DAG as
    8-wave cooperative tiles."""
    import torch
    import paper_2408_09662_amd as xg
    from paper_2408_09662_amd.warm import BATCH_KEYS, batch_programs
    from workloads import configs
    keys = BATCH_KEYS
    xin_host = [configs.item_inputs(k) for k in keys]
    ntot = sum(x[0].shape[1] for x in xin_host)
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

    res = {"instances": ntot}
    progs = batch_programs()
    xin = [[torch.from_numpy(x).to(p.torch_dtype).cuda() for x in xs]
           for p, xs in zip(progs, xin_host)]
    outs = [p.alloc_outputs(x[0].shape[1]) for p, x in zip(progs, xin)]
    runs = [p.bind_eval(x, o) for p, x, o in zip(progs, xin, outs)]
    t_seq = timed(lambda: [r() for r in runs], steps)
    b = xg.Batch(progs)
    ws = b.workspace([x[0].shape[1] for x in xin])
    t_batch = timed(lambda: b.eval(xin, outs, workspace=ws), steps)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = b.capture(xin, outs, stream=s, workspace=ws)
        t_graph = timed(lambda: g.launch(stream=s), steps)
    res["sequential_ms"] = t_seq * 1e3
    res["persistent_ms"] = t_batch * 1e3
    res["persistent_graph_ms"] = t_graph * 1e3
    res["instance_evals_per_s_persistent"] = ntot / t_batch
    # the launch-bound member alone: one lane per instance (8 waves) vs
    # 8-wave cooperative tiles (64 waves)
    k5 = BATCH_KEYS.index("rdag1e5")
    r5w = None
    for w in (1, 8):
        p5 = xg.Program(configs.program_path("rdag1e5"), waves=w)
        x5 = [x.clone() for x in xin[k5]]
        o5 = p5.alloc_outputs(x5[0].shape[1])
        r5 = p5.bind_eval(x5, o5)
        res[f"rdag1e5_n512_waves{w}_ms"] = timed(r5, steps) * 1e3
        r5w = (p5, x5, o5)
    # the same four programs as two concurrent launches: the other three in
    # one persistent launch on one stream, the 1e5-op DAG as 8-wave tiles on
    # a second stream (both default priority), joined by an event
    rest = [i for i in range(len(keys)) if i != k5]
    b3 = xg.Batch([progs[i] for i in rest])
    x3 = [xin[i] for i in rest]
    o3 = [outs[i] for i in rest]
    ws3 = b3.workspace([x[0].shape[1] for x in x3])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    run5 = r5w[0].bind_eval(r5w[1], r5w[2], stream=s2)

    def concurrent():
        cur = torch.cuda.current_stream()
        s1.wait_stream(cur)
        s2.wait_stream(cur)
        b3.eval(x3, o3, workspace=ws3, stream=s1)
        run5()
        cur.wait_stream(s1)
        cur.wait_stream(s2)
    res["concurrent_two_streams_ms"] = timed(concurrent, steps) * 1e3
    # one persistent launch again, with the 1e5-op DAG as 8-wave cooperative
    # tiles and every program on 512-lane workgroups
    from paper_2408_09662_amd.warm import coop_batch_programs
    pc = coop_batch_programs()
    bc = xg.Batch(pc)
    outc = [p.alloc_outputs(x[0].shape[1]) for p, x in zip(pc, xin)]
    wsc = bc.workspace([x[0].shape[1] for x in xin])
    t_coop = timed(lambda: bc.eval(xin, outc, workspace=wsc), steps)
    with torch.cuda.stream(s):
        gc = bc.capture(xin, outc, stream=s, workspace=wsc)
        t_coop_graph = timed(lambda: gc.launch(stream=s), steps)
    # the library's batch autotuner choosing the arrangement itself
    bt = xg.autotune_batch(progs, xin)
    outt = [p.alloc_outputs(x[0].shape[1]) for p, x in zip(progs, xin)]
    wst = bt.workspace([x[0].shape[1] for x in xin])
    res["persistent_autotuned_ms"] = timed(lambda: bt.eval(xin, outt, workspace=wst), steps) * 1e3
    with torch.cuda.stream(s):
        gt = bt.capture(xin, outt, stream=s, workspace=wst)
        res["persistent_autotuned_graph_ms"] = timed(lambda: gt.launch(stream=s), steps) * 1e3
    res["autotuned_block"] = bt.block
    res["instance_evals_per_s_persistent_autotuned_graph"] = ntot / (res["persistent_autotuned_graph_ms"] * 1e-3)
    res["persistent_coop_ms"] = t_coop * 1e3
    res["persistent_coop_graph_ms"] = t_coop_graph * 1e3
    res["instance_evals_per_s_persistent_coop"] = ntot / t_coop
    return res


def bench_rollout(steps=200, tune=True):
    """Quadcopter closed-loop LQR rollouts: 10,000 environments, `steps`
    closed-loop steps per replay -- graph replay vs eager launches."""
    import torch
    import paper_2408_09662_amd as xg
    from workloads import configs
    prog = xg.Program(configs.program_path("quad"))
    z, th = configs.item_inputs("quad")
    n = z.shape[1]
    tz = torch.from_numpy(z).cuda()
    tth = torch.from_numpy(th).cuda()
    plan = xg.autotune(prog, [tz, tth]) if tune else None
    s0, s1 = tz.clone(), torch.empty_like(tz)
    ws = prog.workspace(n, 0)
    runs = [prog.bind_eval([s0, tth], [s1], workspace=ws), prog.bind_eval([s1, tth], [s0], workspace=ws)]
    for k in range(4):
        runs[k & 1]()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        runs[k & 1]()
    e1.record()
    torch.cuda.synchronize()
    t_eager = e0.elapsed_time(e1) * 1e-3
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        g = xg.capture_rollout(prog, s0, s1, [tth], steps, stream=st, workspace=ws)
        g.launch(stream=st)
        st.synchronize()
        e0.record(st)
        g.launch(stream=st)
        e1.record(st)
        st.synchronize()
    t_graph = e0.elapsed_time(e1) * 1e-3
    ops = _ops_per_instance(configs.program_path("quad"))
    return {"environments": n, "steps": steps, "ops_per_step": ops, "plan": _plan_of(prog, plan),
            "eager_s": t_eager, "graph_s": t_graph,
            "env_steps_per_s_graph": n * steps / t_graph,
            "frac_fp64": ops * n * steps / t_graph / PEAK_FP64}


def ldl_sweep(steps):
    """The paper's benchmark axes: LDL^T solves of SPD systems in five sizes
    (operation counts ~10x apart) over batch sizes 1e1..1e5.  Per point: GPU
    time with inputs resident in HBM, GPU time including the host->device
    copy of the inputs and the device->host copy of the outputs (pinned host
    buffers), and the oracle's time on 1 host thread and on all host threads
    (measured on a bounded sample of instances, scaled to the batch)."""
    import torch
    import paper_2408_09662_amd as xg
    from oracle.pyoracle import Program as OProg
    from workloads import configs
    threads = max(1, min(os.cpu_count() or 1, 16))
    rows = []
    for key in configs.LDL_SWEEP:
        path = configs.program_path(key)
        prog = xg.Program(path)
        oprog = OProg(path)
        ops = _ops_per_instance(path)
        nmax = max(configs.LDL_BATCHES)
        host = [torch.from_numpy(a) for a in configs.item_inputs(key, nmax)]
        # oracle rate (instances/s) on a sample taking >= 0.2 s
        cpu = {}
        for th in (1, threads):
            cnt = 16
            while True:
                xs = [a[:, :cnt].numpy().copy() for a in host]
                t0 = time.perf_counter()
                oprog.evaluate(xs, 64, threads=th)
                el = time.perf_counter() - t0
                if el >= 0.2 or cnt >= nmax:
                    break
                cnt = min(nmax, cnt * 4)
            cpu[th] = (cnt / el, cnt)
        for nb in configs.LDL_BATCHES:
            xin = [h[:, :nb].cuda() for h in host]
            hin = [h[:, :nb].contiguous().pin_memory() for h in host]
            out = prog.alloc_outputs(nb)
            hout = [torch.empty(o.shape, dtype=o.dtype).pin_memory() for o in out]
            reps = max(3, min(steps, int(2e9 / max(1, ops * nb))))
            t_res, _ = time_eval(prog, xin, reps, 2)
            run = prog.bind_eval(xin, out)
            for _ in range(2):
                run()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                for d, h in zip(xin, hin):
                    d.copy_(h, non_blocking=True)
                run()
                for h, d in zip(hout, out):
                    h.copy_(d, non_blocking=True)
            e1.record()
            torch.cuda.synchronize()
            t_xfer = e0.elapsed_time(e1) * 1e-3 / reps
            c1 = nb / cpu[1][0]
            ca = nb / cpu[threads][0] if nb >= threads else c1
            rows.append({"function": key, "ops_per_instance": ops, "batch": nb,
                         "gpu_resident_s": t_res, "gpu_with_transfer_s": t_xfer,
                         "cpu_1thread_s": c1, "cpu_all_threads_s": ca,
                         "speedup_vs_serial": c1 / t_res,
                         "speedup_vs_serial_with_transfer": c1 / t_xfer,
                         "speedup_vs_parallel": ca / t_res,
                         "cpu_sample_instances": {1: cpu[1][1], threads: cpu[threads][1]}})
            del xin, hin, out, hout
        del host
    return {"metric": "LDL^T-solve family: time per batch, GPU vs oracle CPU", "threads": threads,
            "rows": rows}


def _host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(path, x, min_seconds=3.0):
    """The oracle (test infrastructure) on the host cores: double precision
    interpreter over the same program and inputs; also on one core, on the
    first 1,024 instances."""
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
    x1 = np.ascontiguousarray(x[:, :1024])
    reps1 = 0
    t1 = time.perf_counter()
    while True:
        o.evaluate([x1], 64, threads=1)
        reps1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= 1.0:
            break
    return {"value": reps * n / el, "unit": "instance-evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"full workload ({n} instances, fp64 interpreter) x {reps} repetitions, "
                      f"{el:.1f} s wall on {threads} threads",
            "value_1_core": reps1 * x1.shape[1] / el1,
            "host": f"{_host_cpu()}, {os.cpu_count()} logical CPUs visible",
            "paper_table_i_speedups_context": PAPER_TABLE_I}


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
    ap.add_argument("--sweep", choices=["ldl"], default=None,
                    help="print the LDL^T-family batch sweep instead of the headline line")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the default launch plan instead of the autotuned one")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only time the fused forward+adjoint kernel at 65,536 instances (profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--only", default=None,
                    help="only time the tuned forward kernel of this workload (e.g. mpc, mpc_mixed, "
                         "pend7_f32) at its instance count or --n, for profiling")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this evaluator runs on one GPU; runs on more than one GPU are not "
              "supported (instances would shard over GPUs with no communication)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2408_09662_amd as xg
    from workloads import configs
    if args.copy_calibration:
        # counter calibration: the copy probe (one 8-byte load and one 8-byte
        # store per lane, as every program argument is accessed) moving a
        # known number of bytes each way
        from workloads import probes
        nb = args.copy_calibration << 20
        cp = xg.Program(probes.copy(1))
        a = torch.empty((1, nb // 8), dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            cp.eval([a], [b])
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": nb, "launches": 5, "kernel": "xg_m0_c0 (copy probe)"}))
        return

    if args.only:
        it = configs.ITEMS[args.only]
        nn = args.n if args.n > 0 else it.n
        po = xg.Program(configs.program_path(args.only))
        xo = [torch.from_numpy(x).to(po.torch_dtype).cuda() for x in it.make_inputs(nn)]
        plo = xg.autotune(po, xo) if not args.no_tune else None
        so, _ = time_eval(po, xo, args.steps, args.warmup)
        opso = _ops_per_instance(configs.program_path(args.only))
        peak = PEAK_FP32 if po.dtype == "f32" else PEAK_FP64
        print(json.dumps({"workload": args.only, "n": nn, "ms_per_eval": so * 1e3,
                          "instance_evals_per_s": nn / so, "ops_per_instance": opso,
                          "frac_of_vector_peak": opso * nn / so / peak, "plan": _plan_of(po, plo),
                          "info": {k: po.info(0)[k] for k in ("n_chunks", "n_ws_slots", "n_lds_slots",
                                                                "vgprs", "scratch_bytes")},
                          "code_hash": f"{po.info(0)['code_hash']:#018x}"}))
        return
    if args.sweep == "ldl":
        print(json.dumps(ldl_sweep(max(3, args.steps // 100))))
        return
    if args.adjoint_only:
        # the fused forward+adjoint kernel alone (tuned plan), for profiling
        p = xg.Program(configs.program_path("pend7_grad"))
        xa = [torch.from_numpy(configs.item_inputs("pend7_grad")[0]).cuda()]
        seeds = [2.0 * p.eval(xa)[0]]
        aplan = xg.autotune_adjoint(p, xa, seeds, fused=True) if not args.no_tune else None
        t = time_adjoint(p, xa, seeds, args.steps, args.warmup, fused=True)
        print(json.dumps({"kernel": "pendulum fused forward+adjoint, fp64", "n": xa[0].shape[1],
                          "ms": t * 1e3, "plan": _plan_of(p, aplan, mode=2),
                          "workspace_slots": p.info(2)["n_ws_slots"]}))
        return

    key = "pend7"
    it = configs.ITEMS[key]
    path = configs.program_path(key)
    n = args.n if args.n > 0 else it.n
    x = it.make_inputs(n)[0]
    prog = xg.Program(path)
    xin = [torch.from_numpy(x).cuda()]
    plan = xg.autotune(prog, xin) if not args.no_tune else None
    prog.compile(0)
    sec, wall = time_eval(prog, xin, args.steps, args.warmup)
    ops = _ops_per_instance(path)
    flops = ops * n
    nbytes = (14 + 14) * 8 * n
    achieved = flops / sec
    value = n / sec
    code_hash = prog.info(0)["code_hash"]
    traffic = PROFILED_TRAFFIC.get(code_hash) if n == PROFILED_N else None
    hw_flops = PROFILED_FLOPS.get(code_hash) if n == PROFILED_N else None
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
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3, copy-calibrated)",
                     "kernel": "xg_m0_c0 (pendulum RK4 forward)",
                     "code_hash": f"{code_hash:#018x}",
                     "algorithmic_flops_per_launch": flops,
                     "algorithmic_bytes_per_launch": nbytes,
                     "issue_frac": flops / sec / PEAK_ISSUE,
                     "counter_fp64_flops_per_launch": hw_flops,
                     "counter_fp64_frac": hw_flops / sec / PEAK_FP64 if hw_flops else None,
                     "issue_note": "IR operations per second over the VALU lane-instruction issue "
                                   "rate (each operation needs at least one lane-instruction "
                                   "unless contracted into an FMA)"},
        "plan": _plan_of(prog, plan),
    }
    out["launch_ms"] = launch_spread(prog, xin, 200)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(path, x)
        out["cpu_baseline"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
        out["cpu_baseline"]["gpu_over_cpu_note"] = (
            "this GPU over the oracle on all listed host cores, inputs resident in HBM (compute only); "
            "the paper's Table I ratios are GPU over parallel CPU code on its own machine")
    if not args.no_secondary:
        sec2 = {}
        steps2 = max(20, args.steps // 10)
        # same program at 4x the instances (fills every SIMD once)
        x4 = configs.ITEMS["pend7_grad"].make_inputs(65536)[0]
        p4 = xg.Program(path)
        x4in = [torch.from_numpy(x4).cuda()]
        plan4 = xg.autotune(p4, x4in) if not args.no_tune else None
        s4, _ = time_eval(p4, x4in, steps2, 5)
        sec2["pendulum7_fwd_f64_n65536"] = {"instance_evals_per_s": 65536 / s4,
                                            "frac_fp64": ops * 65536 / s4 / PEAK_FP64,
                                            "issue_frac": ops * 65536 / s4 / PEAK_ISSUE,
                                            "plan": _plan_of(p4, plan4)}
        # workload 1: the 200-op random DAG at 1,000 instances (16 tiles):
        # launch- and latency-bound, reported per call (autotuned: short
        # phased cooperative tiles spread each tile over several waves)
        pr = xg.Program(configs.program_path("rdag200"))
        xr = [torch.from_numpy(configs.item_inputs("rdag200")[0]).cuda()]
        planr = xg.autotune(pr, xr) if not args.no_tune else None
        sr, _ = time_eval(pr, xr, max(100, steps2), 10)
        # the floor of the same launch path: a program with the same argument
        # shapes (8 inputs, 4 outputs, 1,000 instances) and no arithmetic
        from workloads import probes
        pf = xg.Program(probes.copy(8, 4))
        sf, _ = time_eval(pf, xr, max(100, steps2), 10)
        sec2["rdag200_fwd_f64_n1000"] = {"us_per_call": sr * 1e6, "instance_evals_per_s": 1000 / sr,
                                         "ops_per_instance": _ops_per_instance(configs.program_path("rdag200")),
                                         "plan": _plan_of(pr, planr),
                                         "launch_floor_us_per_call": sf * 1e6,
                                         "launch_floor_note": "copy probe with the same argument "
                                                              "shapes, back-to-back launches"}
        p32 = xg.Program(configs.program_path("pend7_f32"))
        x32 = [torch.from_numpy(x).float().cuda()]
        plan32 = xg.autotune(p32, x32) if not args.no_tune else None
        s32, _ = time_eval(p32, x32, steps2, 5)
        sec2["pendulum7_fwd_f32_n16384"] = {"instance_evals_per_s": n / s32,
                                            "frac_fp32": ops * n / s32 / PEAK_FP32,
                                            "plan": _plan_of(p32, plan32)}
        try:
            ya = torch.from_numpy(2.0 * x).cuda()
            aplan = xg.autotune_adjoint(prog, xin, [ya], fused=True) if not args.no_tune else None
            sa = time_adjoint(prog, xin, [ya], steps2, 5, fused=True)
            sb = time_adjoint(prog, xin, [ya], steps2, 5, fused=False)
            sec2["pendulum7_fused_fwd_adjoint_f64_n16384"] = {"instance_evals_per_s": n / sa,
                                                              "ratio_to_forward": sa / sec,
                                                              "fused_ms": sa * 1e3,
                                                              "separate_fwd_plus_bwd_ms": (sec + sb) * 1e3,
                                                              "adjoint_plan": _plan_of(prog, aplan, mode=2)}
            # the headline launch replayed from a HIP graph vs launched eagerly
            outs_g = prog.alloc_outputs(n)
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                gr = xg.capture_eval(prog, xin, outs_g, stream=st)
                for _ in range(5):
                    gr.launch(stream=st)
                st.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(st)
                for _ in range(args.steps):
                    gr.launch(stream=st)
                e1.record(st)
                st.synchronize()
            sec2["pendulum7_graph_replay_n16384"] = {"graph_ms": e0.elapsed_time(e1) / args.steps,
                                                     "eager_ms": sec * 1e3}
        except Exception as e:  # noqa: BLE001
            sec2["pendulum7_fused_fwd_adjoint_f64_n16384"] = {"error": str(e)[:200]}
        try:
            sec2["pendulum7_reverse_mode_n65536"] = bench_reverse_mode(steps2, tune=not args.no_tune)
        except Exception as e:  # noqa: BLE001
            sec2["pendulum7_reverse_mode_n65536"] = {"error": str(e)[:200]}
        try:
            xm = configs.item_inputs("mpc")[0]
            xmg = [torch.from_numpy(xm).cuda()]
            sweep = {}
            for key in configs.MPC_SWEEP + ["mpc_mixed"]:
                pm = xg.Program(configs.program_path(key))
                planm = xg.autotune(pm, xmg) if not args.no_tune else None
                sm, _ = time_eval(pm, xmg, max(10, steps2 // 4), 3)
                mops = _ops_per_instance(configs.program_path(key))
                sweep[key] = {"instance_evals_per_s": 4096 / sm, "ms_per_eval": sm * 1e3,
                              "ops_per_instance": mops, "frac_fp64": mops * 4096 / sm / PEAK_FP64}
                sweep[key]["plan"] = _plan_of(pm, planm)
            sec2["cartpole_mpc_f64_n4096"] = sweep.pop("mpc")
            sec2["cartpole_mpc_mixed_n4096"] = sweep.pop("mpc_mixed")
            sec2["cartpole_mpc_mixed_n4096"]["speedup_vs_f64"] = (
                sec2["cartpole_mpc_f64_n4096"]["ms_per_eval"] / sec2["cartpole_mpc_mixed_n4096"]["ms_per_eval"])
            sec2["cartpole_mpc_iteration_sweep_n4096"] = sweep
            # the same program with enough instances to fill every SIMD once
            pmb = xg.Program(configs.program_path("mpc"))
            xmb = [torch.from_numpy(configs.ITEMS["mpc"].make_inputs(65536)[0]).cuda()]
            planb = xg.autotune(pmb, xmb) if not args.no_tune else None
            smb, _ = time_eval(pmb, xmb, max(5, steps2 // 8), 2)
            pmm = xg.Program(configs.program_path("mpc_mixed"))
            planmm = xg.autotune(pmm, xmb) if not args.no_tune else None
            smm, _ = time_eval(pmm, xmb, max(5, steps2 // 8), 2)
            sec2["cartpole_mpc_mixed_n65536"] = {"instance_evals_per_s": 65536 / smm,
                                                 "ms_per_eval": smm * 1e3,
                                                 "speedup_vs_f64": smb / smm,
                                                 "plan": _plan_of(pmm, planmm)}
            sec2["cartpole_mpc_f64_n65536"] = {"instance_evals_per_s": 65536 / smb,
                                               "ms_per_eval": smb * 1e3,
                                               "plan": _plan_of(pmb, planb),
                                               "frac_fp64": _ops_per_instance(configs.program_path("mpc")) * 65536 / smb / PEAK_FP64}
        except Exception as e:  # noqa: BLE001
            sec2["cartpole_mpc_f64_n4096"] = {"error": str(e)[:200]}
        try:
            sec2["quadcopter_lqr_rollout"] = bench_rollout(tune=not args.no_tune)
        except Exception as e:  # noqa: BLE001
            sec2["quadcopter_lqr_rollout"] = {"error": str(e)[:300]}
        if not args.no_batch:
            try:
                sec2["uneven_batch"] = bench_batch(steps2)
            except Exception as e:  # noqa: BLE001
                sec2["uneven_batch"] = {"error": str(e)[:300]}
        try:
            out["achievable"] = achievable_peaks(max(10, steps2 // 4))
        except Exception as e:  # noqa: BLE001
            out["achievable"] = {"error": str(e)[:200]}
        out["secondary"] = sec2
    print(json.dumps(out))


if __name__ == "__main__":
    main()
