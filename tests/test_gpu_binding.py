"""GPU tests of the binding's argument checks and of the lifetime rule for
captured graphs (through the C ABI)."""

import ctypes

import numpy as np
import pytest

from workloads import configs, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def xgmod():
    import paper_2408_09662_amd as xg
    return xg


def test_wrong_shapes_rejected_before_any_launch():
    xg = xgmod()
    p = xg.Program(configs.program_path("pend7"))
    n = 256
    x = torch.from_numpy(inputs.pendulum_state(7, 7, n)).cuda()
    out = torch.full((14, n), 7.0, dtype=torch.float64, device="cuda")
    short = torch.zeros((13, n), dtype=torch.float64, device="cuda")
    with pytest.raises(xg.XgError, match="has 13 rows"):
        p.eval([short], [out])
    with pytest.raises(xg.XgError, match="has 13 rows"):
        p.eval([x], [out[:13]])
    with pytest.raises(xg.XgError, match="expected 1 output"):
        p.eval([x], [out, out])
    with pytest.raises(xg.XgError, match="has 13 rows"):
        p.eval_adjoint([x], [short])
    with pytest.raises(xg.XgError, match="has 13 rows"):
        p.eval_adjoint([x], [out], grads=[short])
    with pytest.raises(xg.XgError, match="N >= 256"):
        p.eval([x], [out[:, :100]], n=n)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)  # nothing was launched
    b = xg.Batch([p, xg.Program(configs.program_path("rdag200"))])
    with pytest.raises(xg.XgError, match="2 input and 2 output"):
        b.eval([[x]], [[out]])


def test_retune_refused_while_a_graph_lives(tmp_path, monkeypatch):
    xg = xgmod()
    monkeypatch.setenv("XG_CACHE_DIR", str(tmp_path))
    p = xg.Program(configs.program_path("rdag200"))
    n = 1000
    x = torch.from_numpy(inputs.uniform(101, 8, n)).cuda()
    ref = p.eval([x])[0]
    out = p.alloc_outputs(n)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = xg.capture_eval(p, [x], out, stream=s)
    with pytest.raises(xg.XgError, match="captured graph"):
        xg.autotune(p, [x])
    out[0].fill_(float("nan"))
    g.launch(stream=s)
    s.synchronize()
    assert torch.equal(out[0], ref)  # the graph's kernels are still loaded
    del g
    xg.autotune(p, [x])  # allowed again once the graph is gone
    torch.cuda.synchronize()


def test_program_freed_before_its_graph_stays_loaded():
    """xg_program_free on a program with a live graph defers the unload to
    the graph's free; the graph keeps launching correct code meanwhile."""
    xg = xgmod()
    L = xg.lib()
    p = xg.Program(configs.program_path("pend7"))
    n = 2048
    x = torch.from_numpy(inputs.pendulum_state(3, 7, n)).cuda()
    ref = p.eval([x])[0]
    out = p.alloc_outputs(n)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = xg.capture_eval(p, [x], out, stream=s)
    g._keep = (x, out)  # drop the binding's reference to the program ...
    h, p._h = p._h, None
    L.xg_program_free(h)  # ... and free it through the C ABI while the graph lives
    del p
    for _ in range(3):
        out[0].fill_(float("nan"))
        g.launch(stream=s)
        s.synchronize()
        assert torch.equal(out[0], ref)
    del g  # the last graph frees the program
    torch.cuda.synchronize()
