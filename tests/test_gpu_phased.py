"""GPU parity of phased cooperative tiles (waves > 1, coop_phase > 0): the
waves of one workgroup evaluate the same 64 instances, each running its own
share of the program (in-tree clusters, cheap shared values recomputed per
wave) with a few workgroup barriers; values another wave needs pass through
LDS exchange slots (workspace slots once the LDS allowance is used up).  Checked against the oracle on ragged instance counts,
down to a single instance (one valid lane per wave)."""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [("pend7", 4, 300, 224, 1000), ("pend7", 4, 150, 112, 130), ("pend7", 2, 300, 224, 777),
         ("pend7", 4, 600, 224, 1), ("pend7_f32", 4, 300, 224, 1000), ("quad", 4, 300, 224, 333),
         ("rdag1e3", 2, 150, 112, 65), ("rdag200", 4, 50, 112, 1000), ("rdag200", 2, 50, 112, 37),
         # more exchanged values than LDS slots: the overflow goes through
         # workspace slots
         ("mpc", 2, 300, 168, 333), ("mpc", 4, 150, 112, 130)]


def _run(key, waves, phase, rb, n):
    import paper_2408_09662_amd as xg
    path = configs.program_path(key)
    p = xg.Program(path, waves=waves, coop_phase=phase, reg_budget=rb)
    xs = configs.ITEMS[key].make_inputs(n)
    tdt = p.torch_dtype
    print(f"phased: {key} waves={waves} phase={phase} reg={rb} n={n}", flush=True)
    ys = p.eval([torch.from_numpy(x).to(tdt).cuda() for x in xs])
    torch.cuda.synchronize()
    return p, path, xs, [y.double().cpu().numpy() for y in ys]


@pytest.mark.parametrize("key,waves,phase,rb,n", CASES)
def test_phased_tile_parity(key, waves, phase, rb, n):
    p, path, xs, ys = _run(key, waves, phase, rb, n)
    o = OProg(path)
    if p.dtype == "f64":
        tol = parity.TOL_F64_MPC if key.startswith("mpc") else parity.TOL_F64
        ref = o.evaluate(xs, threads=8)
    else:
        xs32 = [x.astype(np.float32).astype(np.float64) for x in xs]
        ref = o.evaluate(xs32, 64, threads=8)
        tol = parity.f32_tol(o, xs32)
    rep = parity.report(ys, ref, tol)
    assert rep["max"] <= tol, rep
    assert p.info(0)["n_chunks"] == 1


def test_phased_tile_graph_replay():
    import paper_2408_09662_amd as xg
    path = configs.program_path("pend7")
    p = xg.Program(path, waves=4, coop_phase=300, reg_budget=224)
    xs = configs.ITEMS["pend7"].make_inputs(700)
    xin = [torch.from_numpy(x).cuda() for x in xs]
    ref = p.eval(xin)[0].clone()
    out = p.alloc_outputs(700)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = xg.capture_eval(p, xin, out, stream=s)
        for _ in range(3):
            out[0].zero_()
            g.launch(stream=s)
            s.synchronize()
            assert torch.equal(out[0], ref)


def test_phased_tiles_two_per_cu_at_full_size():
    # 2-wave MPC tiles with spill regions small enough that two tiles share
    # a CU (34 LDS slots per lane), at more than one tile per SIMD and a
    # ragged tail: sampled instances (first tiles, the middle, the tail)
    # against the oracle
    import paper_2408_09662_amd as xg
    path = configs.program_path("mpc")
    n = 65536 + 45
    p = xg.Program(path, waves=2, coop_phase=300, reg_budget=168, lds_slots=34)
    x = configs.ITEMS["mpc"].make_inputs(n)[0]
    print(f"phased: mpc waves=2 phase=300 reg=168 lds=34 n={n}", flush=True)
    y = p.eval([torch.from_numpy(x).cuda()])[0].cpu().numpy()
    rng = np.random.default_rng(7)
    idx = np.unique(np.r_[0:64, 32768:32832, n - 109:n, rng.integers(0, n, 160)])
    ref = OProg(path).evaluate([np.ascontiguousarray(x[:, idx])], threads=8)[0]
    rep = parity.report([y[:, idx]], [ref], parity.TOL_F64_MPC)
    assert rep["max"] <= parity.TOL_F64_MPC, rep
    inf = p.info(0)
    assert inf["n_chunks"] == 1 and inf["lds_bytes"] <= 80 * 1024
