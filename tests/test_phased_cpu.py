"""Host checks of phased cooperative-tile plans (no GPU): plans form for
narrow programs at several wave counts and phase lengths, and in the
generated kernel every wave's branch passes the same number of workgroup
barriers with no early exit (a wave that skipped a barrier would leave the
others waiting)."""

import os
import re
import subprocess
import sys

import pytest

import paper_2408_09662_amd as xg
from workloads import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("key,waves,phase", [("pend7", 2, 150), ("pend7", 4, 300), ("pend7", 4, 600),
                                             ("pend7_f32", 4, 300), ("quad", 4, 300), ("rdag200", 2, 50)])
def test_phased_plan_forms(key, waves, phase):
    p = xg.Program(configs.program_path(key), waves=waves, coop_phase=phase, reg_budget=224)
    inf = p.info(0)
    assert inf["n_chunks"] == 1
    assert inf["n_ops"] > 0


def _branches(src):
    body = src[src.index("if (xg_w == 0) {"):]
    parts = re.split(r"\n  (?:else )?if \(xg_w == \d+\) \{\n", "\n" + body)
    return [p for p in parts if p.strip()]


@pytest.mark.slow
def test_every_wave_passes_the_same_barriers(tmp_path):
    code = (
        "import paper_2408_09662_amd as xg\n"
        "from workloads import configs\n"
        "for w, ph in ((4, 300), (2, 150)):\n"
        "    xg.Program(configs.program_path('pend7'), waves=w, coop_phase=ph, reg_budget=224).precompile(0)\n")
    env = dict(os.environ, XG_DUMP_DIR=str(tmp_path), XG_CACHE_DIR=str(tmp_path / "cache"))
    subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, check=True)
    srcs = [open(os.path.join(tmp_path, f)).read() for f in os.listdir(tmp_path) if f.endswith(".hip")]
    assert len(srcs) == 2
    for s in srcs:
        m = re.search(r"phased cooperative tile of (\d+) waves, (\d+) phases", s)
        assert m, s[:200]
        w, phases = int(m.group(1)), int(m.group(2))
        br = _branches(s)
        assert len(br) == w
        for b in br:
            assert b.count("xg_barrier();") == phases - 1
            assert "return" not in b
