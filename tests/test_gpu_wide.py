"""GPU parity of cooperative tiles (waves > 1): several waves of one
workgroup evaluate the same 64 instances, the program split by dependency
level, values crossing waves passed through the workspace between
workgroup barriers.  Checked against the oracle on ragged instance counts."""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [("rdag200", 4, 1000), ("rdag200", 16, 65), ("rdag1e4", 4, 1100), ("rdag1e4", 8, 300),
         ("pend7", 2, 777), ("pend7", 4, 130), ("mpc", 4, 333), ("rdag1e5", 16, 100)]


def _run(key, waves, n, **opts):
    import paper_2408_09662_amd as xg
    path = configs.program_path(key)
    p = xg.Program(path, waves=waves, **opts)
    xs = configs.ITEMS[key].make_inputs(n)
    tdt = p.torch_dtype
    ys = p.eval([torch.from_numpy(x).to(tdt).cuda() for x in xs])
    torch.cuda.synchronize()
    return p, path, xs, [y.double().cpu().numpy() for y in ys]


@pytest.mark.parametrize("key,waves,n", CASES)
def test_cooperative_tile_parity(key, waves, n):
    p, path, xs, ys = _run(key, waves, n)
    o = OProg(path)
    if p.dtype == "f64":
        tol = parity.TOL_F64_MPC if key.startswith("mpc") else parity.TOL_F64
        ref = o.evaluate(xs, threads=8)
    else:
        xs32 = [x.astype(np.float32).astype(np.float64) for x in xs]
        ref = o.evaluate(xs32, 64, threads=8)
        e32 = parity.max_err(o.evaluate(xs32, 32, threads=8), ref)
        tol = max(parity.TOL_F32, 4 * e32)
    rep = parity.report(ys, ref, tol)
    assert rep["max"] <= tol, rep
    assert p.info(0)["n_chunks"] == 1


def test_cooperative_tile_graph_replay():
    import paper_2408_09662_amd as xg
    path = configs.program_path("rdag1e4")
    p = xg.Program(path, waves=4)
    xs = configs.ITEMS["rdag1e4"].make_inputs(700)
    xin = [torch.from_numpy(x).float().cuda() for x in xs]
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


def test_batch_rejects_mismatched_workgroup_sizes():
    """A 4-wave cooperative tile needs 256-lane workgroups; a 64-lane
    program cannot share its launch."""
    import paper_2408_09662_amd as xg
    a = xg.Program(configs.program_path("rdag200"), waves=4)
    b = xg.Program(configs.program_path("rdag200"))
    with pytest.raises(xg.XgError):
        xg.Batch([a, b])
