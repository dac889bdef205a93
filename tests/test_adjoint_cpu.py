"""The library's reverse-mode transformation checked on the CPU: the
adjoint program it builds (recursive checkpointing: cuts at small live sets,
recomputation between them) is evaluated by a plain sequential walk of its
nodes (tests/native/adjoint_eval.cpp) and compared with the oracle's
dual-number gradient and forward values.  The GPU tests check the same
programs compiled and run on the device."""

import os
import subprocess

import numpy as np
import pytest

import paper_2408_09662_amd as xg
from oracle.pyoracle import Program as OProg
from tests import parity
from workloads import configs, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = tmp_path_factory.mktemp("adj") / "adjoint_eval"
    libdir = os.path.dirname(xg._abi.LIB_PATH)
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(libdir, "csrc"), os.path.join(ROOT, "tests", "native", "adjoint_eval.cpp"),
                    "-o", str(exe), "-L", libdir, "-l:libxg.so", f"-Wl,-rpath,{libdir}"], check=True)
    return exe


def run_adjoint(exe, path, xs, seeds, seg, fanout, tmp_path):
    d = xg.load_program_file(path)
    desc = tmp_path / "desc.txt"
    prec = d["prec"] if d["prec"] is not None else np.zeros(len(d["instr"]), dtype=np.int8)
    with open(desc, "w") as f:
        f.write(f"{64 if d['dtype'] == 'f64' else 32} {d['n_work']} {len(d['nnz_in'])} "
                + " ".join(map(str, d["nnz_in"])) + f" {len(d['nnz_out'])} " + " ".join(map(str, d["nnz_out"]))
                + f" {len(d['consts'])} " + " ".join(float(c).hex() for c in d["consts"])
                + f" {len(d['instr'])}\n")
        for (op, o, a, b), p in zip(d["instr"], prec):
            f.write(f"{op} {o} {a} {b} {int(p)}\n")
    n = xs[0].shape[1]
    blob = np.concatenate([np.concatenate(xs, axis=0), np.concatenate(seeds, axis=0)], axis=0).T
    inp = tmp_path / "in.bin"
    with open(inp, "wb") as f:
        f.write(np.int64(n).tobytes())
        f.write(np.ascontiguousarray(blob, dtype=np.float64).tobytes())
    outp = tmp_path / "out.bin"
    subprocess.run([str(exe), str(desc), str(seg), str(fanout), str(inp), str(outp)], check=True)
    raw = np.fromfile(outp, dtype=np.float64)
    nrec = int(raw[-1])
    tot_in, tot_out = sum(d["nnz_in"]), sum(d["nnz_out"])
    vals = raw[:-1].reshape(n, tot_in + tot_out).T
    return vals[:tot_in], vals[tot_in:], nrec


@pytest.mark.parametrize("key,seg,fanout", [("pend7", 250, 2), ("pend7", 250, 4), ("pend7", 1500, 4),
                                            ("pend7", 0, 2), ("rdag200", 40, 2), ("rdag200", 40, 3),
                                            ("quad", 500, 2), ("mpc", 2000, 2)])
def test_adjoint_program_matches_dual_numbers(driver, tmp_path, key, seg, fanout):
    path = configs.program_path(key)
    n = 48
    xs = [np.ascontiguousarray(x[:, :n]) for x in configs.item_inputs(key, n)]
    o = OProg(path)
    ys = o.evaluate(xs)
    ybar = [np.random.default_rng(3).normal(size=y.shape) for y in ys]
    g, y, nrec = run_adjoint(driver, path, xs, ybar, seg, fanout, tmp_path)
    _, gr = o.vjp(xs, ybar)
    gr = np.concatenate(gr, axis=0)
    yr = np.concatenate(ys, axis=0)
    tol = parity.TOL_F64_MPC if key == "mpc" else 1e-12
    assert parity.max_err([g], [gr]) <= tol, parity.max_err([g], [gr])
    assert np.array_equal(y, yr)  # the forward sweep is the program itself, op for op
    if seg > 0:
        assert nrec > 0
