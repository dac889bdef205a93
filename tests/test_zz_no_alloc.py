"""xg_eval_adjoint_noalloc: the adjoint whose workspace is the library's
fixed device array, against xg_eval_adjoint with a caller-provided
workspace (same kernels, so the results must be bitwise equal)."""

import numpy as np
import pytest

import paper_2408_09662_amd as xg
from paper_2408_09662_amd._abi import XgError
from workloads import configs, inputs

pytestmark = pytest.mark.gpu


def _case(n, seed):
    import torch
    xs = torch.from_numpy(inputs.pendulum_state(seed, 7, n)).cuda()
    rng = np.random.default_rng(seed + 1)
    seeds = torch.from_numpy(rng.standard_normal((14, n))).cuda()
    return xs, seeds


@pytest.mark.parametrize("fused", [True, False])
def test_noalloc_adjoint_equals_workspace_adjoint(fused):
    import torch
    torch.cuda.set_device(0)
    p = xg.Program(configs.program_path("pend7"))
    mode = 2 if fused else 1
    p.compile(mode)
    # two calls in a row, the second on fewer instances (the array keeps the
    # first call's contents)
    for n, seed in ((4096, 104), (1000, 105)):
        print(f"noalloc adjoint: pend7 mode {mode} n={n} seed={seed}", flush=True)
        xs, seeds = _case(n, seed)
        ref = p.eval_adjoint([xs], [seeds], with_outputs=fused)
        g = [torch.full((14, n), float("nan"), dtype=torch.float64, device="cuda")]
        y = [torch.full((14, n), float("nan"), dtype=torch.float64, device="cuda")] if fused else None
        got = p.eval_adjoint_noalloc([xs], [seeds], g, y)
        torch.cuda.synchronize()
        if fused:
            assert torch.equal(got[0][0], ref[0][0])
            assert torch.equal(got[1][0], ref[1][0])
        else:
            assert torch.equal(got[0], ref[0])


def test_noalloc_adjoint_refuses_unloaded_kernels_and_oversized_n():
    import torch
    torch.cuda.set_device(0)
    p = xg.Program(configs.program_path("pend7"))
    xs, seeds = _case(256, 106)
    g = [torch.empty((14, 256), dtype=torch.float64, device="cuda")]
    with pytest.raises(XgError, match="not loaded on this device"):
        p.eval_adjoint_noalloc([xs], [seeds], g)
    p.compile(1)
    n = 1 << 20  # needs far more than the 128 MiB array
    need = p.workspace_bytes(n, 1)
    assert need > 128 << 20
    xb, sb = _case(n, 107)
    gb = [torch.empty((14, n), dtype=torch.float64, device="cuda")]
    with pytest.raises(XgError, match="fixed scratch array holds"):
        p.eval_adjoint_noalloc([xb], [sb], gb)
    # a refused call leaves the entry point usable
    p.eval_adjoint_noalloc([xs], [seeds], g)
    torch.cuda.synchronize()
    assert torch.equal(g[0], p.eval_adjoint([xs], [seeds])[0])


def test_noalloc_fused_adjoint_at_full_size_in_the_tuned_plan():
    # the array holds the fused adjoint's workspace at 65,536 instances in
    # the plan the adjoint autotuner picks (the benchmark's configuration)
    import torch
    torch.cuda.set_device(0)
    n = 65536
    p = xg.Program(configs.program_path("pend7"))
    xs, seeds = _case(n, 108)
    xg.autotune_adjoint(p, [xs], [seeds], fused=True)
    assert p.workspace_bytes(n, 2) <= 128 << 20  # XG_NOALLOC_SCRATCH_BYTES
    p.compile(2)
    print(f"noalloc adjoint: pend7 mode 2 n={n} (tuned plan)", flush=True)
    ref = p.eval_adjoint([xs], [seeds], with_outputs=True)
    g = [torch.full((14, n), float("nan"), dtype=torch.float64, device="cuda")]
    y = [torch.full((14, n), float("nan"), dtype=torch.float64, device="cuda")]
    got = p.eval_adjoint_noalloc([xs], [seeds], g, y)
    torch.cuda.synchronize()
    assert torch.equal(got[0][0], ref[0][0])
    assert torch.equal(got[1][0], ref[1][0])
