"""GPU parity of the quadcopter closed-loop LQR step and of its
graph-captured rollout (call through the C ABI)."""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _setup(n):
    import paper_2408_09662_amd as xg
    path = configs.program_path("quad")
    z, th = configs.ITEMS["quad"].make_inputs(n)
    return xg, path, z, th


def test_single_step_ragged():
    xg, path, z, th = _setup(1001)
    p = xg.Program(path)
    ys = p.eval([torch.from_numpy(z).cuda(), torch.from_numpy(th).cuda()])
    torch.cuda.synchronize()
    rep = parity.report([ys[0].cpu().numpy()], OProg(path).evaluate([z, th], threads=8),
                        parity.TOL_F64)
    assert rep["max"] <= parity.TOL_F64, rep


@pytest.mark.parametrize("steps", [1, 20])
def test_graph_rollout_matches_eager_and_oracle(steps):
    n = 777
    xg, path, z, th = _setup(n)
    p = xg.Program(path)
    tz = torch.from_numpy(z).cuda()
    tth = torch.from_numpy(th).cuda()
    # eager GPU rollout
    cur = tz.clone()
    for _ in range(steps):
        cur = p.eval([cur, tth])[0]
    # oracle rollout
    o = OProg(path)
    r = z.copy()
    for _ in range(steps):
        r = o.evaluate([r, th], threads=8)[0]
    s = torch.cuda.Stream()
    s0, s1 = tz.clone(), torch.empty_like(tz)
    with torch.cuda.stream(s):
        g = xg.capture_rollout(p, s0, s1, [tth], steps, stream=s)
        for rep in range(2):
            s0.copy_(tz)
            g.launch(stream=s)
            s.synchronize()
            fin = (s0 if steps % 2 == 0 else s1).cpu().numpy()
            assert np.array_equal(fin, cur.cpu().numpy()), f"replay {rep} differs from eager"
    # parity with the oracle's own rollout: per step within 1e-12; the
    # closed loop is contracting, so 20 composed steps stay within 1e-11
    tol = parity.TOL_F64 if steps == 1 else 10 * parity.TOL_F64
    rep = parity.report([fin], [r], tol)
    assert rep["max"] <= tol, rep


def test_rollout_rejects_bad_shapes():
    xg, path, z, th = _setup(64)
    p = xg.Program(path)
    tz = torch.from_numpy(z).cuda()
    s = torch.cuda.Stream()
    with pytest.raises(xg.XgError):
        xg.capture_rollout(p, tz, tz, [torch.from_numpy(th).cuda()], 4, stream=s)
    with pytest.raises(xg.XgError):
        xg.capture_rollout(p, tz, tz.clone(), [torch.from_numpy(th).cuda()], 0, stream=s)
