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


def _lds_accesses(src):
    """(base name, constant) of every LDS access in a generated source."""
    return re.findall(r"xg_lds_(?:ld|st)\((xg_[lx]b\d+), (\d+)u", src)


@pytest.mark.slow
def test_lds_constants_fit_the_offset_field(tmp_path):
    # a phased tile whose exchange area exceeds 64 KiB and a single-wave
    # kernel whose spill region does: every LDS access names a base the
    # kernel defines and a constant the instruction's 16-bit offset holds
    code = (
        "import paper_2408_09662_amd as xg\n"
        "from workloads import configs\n"
        "xg.Program(configs.program_path('pend7'), waves=4, coop_phase=300, reg_budget=168, lds_slots=79).precompile(0)\n"
        "xg.Program(configs.program_path('pend7'), reg_budget=48, lds_slots=300).precompile(0)\n")
    env = dict(os.environ, XG_DUMP_DIR=str(tmp_path), XG_CACHE_DIR=str(tmp_path / "cache"))
    subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, check=True)
    srcs = [open(os.path.join(tmp_path, f)).read() for f in os.listdir(tmp_path) if f.endswith(".hip")]
    assert len(srcs) == 2
    seen_high = set()
    for s in srcs:
        acc = _lds_accesses(s)
        assert acc, "no LDS accesses"
        assert "xg_lds_ld(lds" not in s and "xg_lds_st(xch" not in s
        for base, c in acc:
            assert int(c) < 65536, (base, c)
            assert re.search(r"unsigned %s = " % base, s), base
            if not base.endswith("0"):
                seen_high.add(base[:5])
    # both kinds of region reach past 64 KiB: the exchange area of the
    # tile and the spill region of the single wave
    assert seen_high == {"xg_xb", "xg_lb"}


@pytest.mark.slow
def test_phased_tiles_in_a_batch_pass_the_same_barriers(tmp_path):
    # a persistent batch holding a phased program: in its run() every wave
    # branch passes the same number of barriers, with no early exit, and the
    # batch's LDS array holds the exchange slots and spill regions
    code = (
        "import paper_2408_09662_amd as xg\n"
        "from workloads import configs\n"
        "a = xg.Program(configs.program_path('rdag1e3'), waves=2, coop_phase=150, reg_budget=112)\n"
        "b = xg.Program(configs.program_path('rdag200'), waves=2)\n"
        "xg.Batch([a, b])\n")
    env = dict(os.environ, XG_DUMP_DIR=str(tmp_path), XG_CACHE_DIR=str(tmp_path / "cache"))
    subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, check=True)
    srcs = [open(os.path.join(tmp_path, f)).read() for f in os.listdir(tmp_path) if f.endswith(".hip")]
    batch = [s for s in srcs if "persistent batch" in s[:200]]
    assert len(batch) == 1
    s = batch[0]
    assert "#define xg_barrier() __syncthreads()" in s
    r = s.index("void run(long long ibase, int xg_w)")  # the first program's run()
    body = s[r:s.index("namespace P1 {", r)]
    parts = re.split(r"\n  (?:else )?if \(xg_w == \d+\) \{\n", "\n" + body)[1:]
    assert len(parts) == 2
    counts = {p.count("xg_barrier();") for p in parts}
    assert len(counts) == 1 and counts.pop() > 0
    assert all("return" not in p for p in parts)
    lds = int(re.search(r"char xg_lds_raw\[(\d+)\]", s).group(1))
    m = re.search(r"lT\* lds = \(lT\*\)xg_lds_raw \+ (\d+) \+ xg_w \* (\d+);", body)
    xch_elems, wave_elems = (int(m.group(1)), int(m.group(2))) if m else (0, 0)
    assert (xch_elems + 2 * wave_elems) * 4 <= lds  # binary32 program
